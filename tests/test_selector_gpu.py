"""The deployed selector on the GPU (section 5.1 and the learned MLP
selector): host and device MLP picks agree; the out-of-range fallback times
the chosen kernels; the validated choice of selector scores each kind the
way the regret oracle does; and, on the committed MI355X timing table, the
trained MLP cost model beats both the single best kernel and decision tree
B on the held-out shapes (what the network gains over the method without
it)."""
import numpy as np
import pytest

import synth
from oracle import regret as oreg

pytestmark = pytest.mark.gpu


def _load(dtype_name="f32"):
    from paper_2008_13145_amd import tune
    T, P, C, meta = tune.load_table(tune.table_path(dtype_name))
    problems = [tuple(int(v) for v in p) for p in P]
    train, test = synth.train_test_split()
    return T, problems, synth.rows_of_shapes(train), synth.rows_of_shapes(test)


def _mlp_ws(kt, torch, n, d, k):
    b = kt.Handle.mlp_workspace_bytes(n, d, k)
    return torch.empty(b, dtype=torch.uint8, device="cuda"), b


CHOSEN8 = [10, 25, 47, 60, 81, 100, 120, 150]


def test_mlp_host_picks_equal_device_picks(gpu, kt):
    h, torch = gpu
    T, problems, tr, te = _load()
    ws, wb = _mlp_ws(kt, torch, len(tr), T.shape[1], 8)
    h.fit_selector(kt.SEL_MLP, [problems[r] for r in tr], T[tr], CHOSEN8, mlp_steps=500,
                   workspace=ws, ws_bytes=wb)
    h.set_fallback(0)
    host = [h.select(*p) for p in problems]
    # kt_shape: four int64 then two int32 (packed here into one int64)
    arr = np.array([[m, n, k, b, (ta | (tb << 32))] for (m, n, k, b, ta, tb) in problems], np.int64)
    d_shapes = torch.from_numpy(arr).cuda()
    d_ids = torch.zeros(len(problems), dtype=torch.int32, device="cuda")
    h.select_batch(d_shapes, len(problems), d_ids)
    torch.cuda.synchronize()
    assert d_ids.cpu().numpy().tolist() == host
    h.set_fallback(1)


def test_fallback_times_the_chosen_kernels_outside_the_box(gpu, kt):
    """Outside the training box the pick is timed among the chosen kernels and
    the split-K variants of their configurations, once, then cached."""
    h, torch = gpu
    T, problems, tr, te = _load()
    shapes = [problems[r] for r in tr]
    h.fit_selector(kt.SEL_DT_B, shapes, T[tr], CHOSEN8)
    info = h.selector_info()
    assert info["fallback"] == 1 and info["box_lo"][0] >= 16
    out = (1, 4096, 25088, 1, 0, 0)          # M = 1 lies below every training M
    h.set_fallback(0)
    model_pick = h.select(*out)
    h.set_fallback(1)
    pick = h.select(*out)
    # a chosen kernel, or a split-K variant of a chosen configuration
    assert pick in CHOSEN8 or h.get_kernel(pick)[1] in CHOSEN8
    assert h.select(*out) == pick            # cached
    inside = problems[tr[0]]
    h.set_fallback(0)
    p0 = h.select(*inside)
    h.set_fallback(1)
    assert h.select(*inside) == p0           # inside the box the model decides
    assert model_pick in CHOSEN8
    # exhaustive fallback: any kernel the library holds, timed once, cached;
    # inside the box the model still decides
    h.set_fallback(2)
    ex = h.select(*out)
    assert 0 <= ex < h.num_kernels()
    assert h.select(*out) == ex
    assert h.select(*inside) == p0
    h.set_fallback(1)


def test_validated_selector_scores_match_the_oracle(gpu, kt):
    h, torch = gpu
    T, problems, tr, te = _load()
    train, _ = synth.train_test_split()
    fit_shapes, val_shapes = synth.train_validation_split(train)
    val_set = set(val_shapes)
    shapes = [problems[r] for r in tr]
    is_val = [synth.shape_of_row(r) in val_set for r in tr]
    assert 0 < sum(is_val) < len(tr)
    ws, wb = _mlp_ws(kt, torch, len(tr), T.shape[1], 8)
    kind, scores = h.fit_selector_validated(shapes, T[tr], CHOSEN8, is_val, mlp_steps=600,
                                            workspace=ws, ws_bytes=wb)
    assert kind == int(np.argmax(scores))
    # the same scores from separate fits, scored by the regret oracle
    fit_rows = [r for r, v in zip(tr, is_val) if not v]
    val_rows = [r for r, v in zip(tr, is_val) if v]
    h2 = kt.Handle(0)
    h2.set_fallback(0)
    for kk in range(4):
        h2.fit_selector(kk, [problems[r] for r in fit_rows], T[fit_rows], CHOSEN8, mlp_steps=600,
                        workspace=ws, ws_bytes=wb)
        picks = [h2.select(*problems[r]) for r in val_rows]
        assert abs(oreg.selected(T, picks, val_rows)["geomean"] - scores[kk]) < 1e-12, kk
    h2.close()
    assert h.selector_info()["kind"] == kind


def test_mlp_gains_over_the_method_without_it(gpu, kt):
    """Trained on the training rows of the committed MI355X table (k-means
    pruning to 8 kernels under the normalization chosen on those rows), the
    MLP cost model keeps more of the optimum on the held-out shapes than the
    best single kernel (no selection) and than decision tree B (the paper's
    selector), each by a stated margin."""
    h, torch = gpu
    T, problems, tr, te = _load()
    pws_b = kt.Handle.prune_workspace_bytes(len(tr), T.shape[1], 8, 10)
    pws = torch.empty(pws_b, dtype=torch.uint8, device="cuda")
    chosen = h.prune_auto(T[tr], 8, seed=synth.SEED, workspace=pws, ws_bytes=pws_b)["chosen"]
    shapes = [problems[r] for r in tr]
    ws, wb = _mlp_ws(kt, torch, len(tr), T.shape[1], 8)
    res = {}
    for kind in (kt.SEL_DT_B, kt.SEL_MLP):
        h.fit_selector(kind, shapes, T[tr], chosen, mlp_steps=3000, workspace=ws, ws_bytes=wb)
        h.set_fallback(0)
        res[kind] = h.evaluate(T, rows=te, picks=[h.select(*problems[r]) for r in te])["geomean"]
        h.set_fallback(1)
    # the best single kernel over the training rows, on the held-out rows
    single = max(range(T.shape[1]), key=lambda c: h.evaluate(T, rows=tr, picks=[c] * len(tr))["geomean"])
    res["single"] = h.evaluate(T, rows=te, picks=[single] * len(te))["geomean"]
    print("held-out geomean: MLP %.4f, DT-B %.4f, single kernel %.4f"
          % (res[kt.SEL_MLP], res[kt.SEL_DT_B], res["single"]), flush=True)
    assert res[kt.SEL_MLP] >= res[kt.SEL_DT_B] + 0.01
    assert res[kt.SEL_MLP] >= res["single"] + 0.05
    assert res[kt.SEL_MLP] >= 0.90
