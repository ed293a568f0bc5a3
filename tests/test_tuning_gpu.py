"""GPU parity of the tuning pipeline: normalization, k-means pruning, Top-N,
batch selection and the MLP cost model's kernels, against the CPU oracle.

Integer steps (normalization, k-means, Top-N, tree walk) must match bit for
bit; MLP gradients (FP32 on the GPU vs FP64 oracle at the same weights) must
agree within 1e-4 relative Frobenius error per parameter tensor."""
import math

import numpy as np
import pytest

import synth
from oracle import cart, kmeans as okm, mlp as omlp, normalize as onz

pytestmark = pytest.mark.gpu


def _planted_table(rng, n_rows, n_cfg, n_groups):
    """Timing table with n_groups families of rows, each fastest on its own
    few configurations; the rest slower by a random factor."""
    T = rng.integers(2000, 200000, size=(n_rows, n_cfg)).astype(np.int64)
    fav = [rng.choice(n_cfg, size=3, replace=False) for _ in range(n_groups)]
    for i in range(n_rows):
        g = i % n_groups
        T[i, fav[g]] = rng.integers(900, 1100, size=3)
    return T


def _draws(seed, n_init, k):
    return okm.restart_draws(synth.SplitMix64, seed, n_init, k)


def test_normalize_all_variants(gpu):
    h, torch = gpu
    rng = np.random.default_rng(1)
    T = rng.integers(1, 10 ** 8, size=(97, 164)).astype(np.int64)
    T[rng.random(T.shape) < 0.05] = -1
    T[3, :] = -1                       # a row with nothing measured
    T[5, :] = 777                      # all tied
    dT = torch.from_numpy(T).cuda()
    for norm in range(4):
        out = torch.zeros(T.shape, dtype=torch.int16, device="cuda")
        h.normalize(dT, T.shape[0], T.shape[1], norm, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint16)
        assert np.array_equal(got, onz.normalize(T, norm)), norm


@pytest.mark.parametrize("k,norm,seed", [(4, 0, 13145), (8, 0, 7), (8, 1, 13145), (5, 2, 3),
                                         (6, 3, 99), (15, 0, 13145)])
def test_prune_kmeans_bitwise(gpu, k, norm, seed):
    kt_mod = __import__("paper_2008_13145_amd")
    h, torch = gpu
    rng = np.random.default_rng(k * 10 + norm)
    T = _planted_table(rng, 960, 164, 9)
    n_init, max_iter = 10, 300
    ws_bytes = kt_mod.Handle.prune_workspace_bytes(960, 164, k, n_init)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    got = h.prune(T, k, norm=norm, seed=seed, n_init=n_init, max_iter=max_iter, workspace=ws,
                  ws_bytes=ws_bytes)
    X = onz.normalize(T, norm)
    ref = okm.kmeans(X, k, _draws(seed, n_init, k), max_iter)
    assert got["inertia"] == ref["inertia"]
    assert np.array_equal(got["labels"], ref["labels"])
    assert np.array_equal(got["centroids"], ref["centroids"])
    assert got["chosen"] == okm.centroids_to_configs(ref["centroids"])


@pytest.mark.parametrize("frac,norm", [(0.1, 0), (0.25, 2), (0.5, 1)])
def test_prune_sparse_table_bitwise(gpu, frac, norm):
    """Pruning from a sparsely measured table (only a random fraction of the
    entries timed; the rest -1, which normalize to 0) still matches the
    oracle bit for bit."""
    kt_mod = __import__("paper_2008_13145_amd")
    h, torch = gpu
    rng = np.random.default_rng(int(frac * 100) + norm)
    T = _planted_table(rng, 960, 164, 9)
    T[rng.random(T.shape) >= frac] = -1
    k, n_init, seed = 8, 10, 13145
    ws_bytes = kt_mod.Handle.prune_workspace_bytes(960, 164, k, n_init)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    got = h.prune(T, k, norm=norm, seed=seed, n_init=n_init, workspace=ws, ws_bytes=ws_bytes)
    ref = okm.kmeans(onz.normalize(T, norm), k, _draws(seed, n_init, k), 300)
    assert got["inertia"] == ref["inertia"]
    assert got["chosen"] == okm.centroids_to_configs(ref["centroids"])


@pytest.mark.parametrize("n,d,k,max_iter", [(5, 3, 3, 300), (7, 4, 1, 300), (6, 6, 6, 300),
                                            (40, 10, 3, 0), (40, 10, 3, 1), (300, 20, 7, 2)])
def test_prune_edge_cases(gpu, n, d, k, max_iter):
    kt_mod = __import__("paper_2008_13145_amd")
    h, torch = gpu
    rng = np.random.default_rng(n + d + k)
    T = rng.integers(100, 400, size=(n, d)).astype(np.int64)
    T[0] = T[1]                        # duplicate rows exercise empty clusters and ties
    ws_bytes = kt_mod.Handle.prune_workspace_bytes(n, d, k, 3)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    got = h.prune(T, k, seed=5, n_init=3, max_iter=max_iter, workspace=ws, ws_bytes=ws_bytes)
    ref = okm.kmeans(onz.normalize(T, 0), k, _draws(5, 3, k), max_iter)
    assert got["inertia"] == ref["inertia"]
    assert np.array_equal(got["labels"], ref["labels"])
    assert np.array_equal(got["centroids"], ref["centroids"])
    assert got["chosen"] == okm.centroids_to_configs(ref["centroids"])


def test_prune_rejects_bad_arguments(gpu):
    kt_mod = __import__("paper_2008_13145_amd")
    h, torch = gpu
    T = np.ones((10, 5), np.int64)
    ws_bytes = kt_mod.Handle.prune_workspace_bytes(10, 5, 3, 2)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    for k in (0, 6, 11):
        with pytest.raises(kt_mod.KtError) as e:
            h.prune(T, k, n_init=2, workspace=ws, ws_bytes=ws_bytes)
        assert e.value.status == -1
    with pytest.raises(kt_mod.KtError) as e:
        h.prune(T, 3, n_init=2, workspace=ws, ws_bytes=16)
    assert e.value.status == -5


def test_topn_matches_oracle(gpu):
    kt_mod = __import__("paper_2008_13145_amd")
    h, torch = gpu
    rng = np.random.default_rng(2)
    T = _planted_table(rng, 500, 164, 12)
    ws_bytes = kt_mod.Handle.prune_workspace_bytes(500, 164, 1, 1)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    for k in (4, 8, 15):
        got = h.prune_topn(T, k, workspace=ws, ws_bytes=ws_bytes)
        assert got == okm.top_n(onz.normalize(T, 0), k)


def test_select_batch_matches_host_walk(gpu):
    h, torch = gpu
    rng = np.random.default_rng(3)
    problems = synth.sweep_problems(100, 555)
    T = _planted_table(rng, len(problems), 40, 6)
    chosen = [2, 11, 30, 7, 19]
    for kind in (0, 1, 2):
        h.fit_selector(kind, problems, T, chosen)
        queries = problems + [(16, 16, 16, 1, 0, 0), (4096, 4096, 4096, 64, 1, 1)]
        arr = np.array([[m, n, k, b, (ta | (tb << 32))] for (m, n, k, b, ta, tb) in queries], np.int64)
        d_shapes = torch.from_numpy(arr).cuda()
        d_ids = torch.zeros(len(queries), dtype=torch.int32, device="cuda")
        h.select_batch(d_shapes, len(queries), d_ids)
        torch.cuda.synchronize()
        # the device walk is the model's pick; compare with the host walk
        # without the out-of-range fallback (the two extra queries lie outside)
        h.set_fallback(0)
        want = [h.select(*q) for q in queries]
        h.set_fallback(1)
        assert d_ids.cpu().tolist() == want
        ref = cart.fit(np.array(problems), cart.labels_from_times(T, chosen), 5,
                       *cart.TREE_PARAMS["ABC"[kind]])
        assert want[:len(problems)] == [chosen[c] for c in cart.predict(ref, np.array(problems))]


def _mlp_data(n, k, seed):
    rng = np.random.default_rng(seed)
    problems = synth.sweep_problems(n // 4 + 1, 900 + seed)[:n]
    X = omlp.features(problems)
    Y = rng.uniform(0, 1, size=(n, k))
    return problems, X, Y


def _pack(p):
    return np.concatenate([p[name].reshape(-1) for name in omlp.PARAM_ORDER]).astype(np.float32)


def _unpack(v, k):
    shapes = {"W1": (64, 6), "b1": (64,), "W2": (64, 64), "b2": (64,), "W3": (k, 64), "b3": (k,)}
    out, o = {}, 0
    for name in omlp.PARAM_ORDER:
        sz = int(np.prod(shapes[name]))
        out[name] = np.asarray(v[o:o + sz], dtype=np.float64).reshape(shapes[name])
        o += sz
    return out


@pytest.mark.parametrize("n,k", [(960, 8), (130, 4), (64, 15)])
def test_mlp_gradients_vs_oracle(gpu, n, k):
    kt_mod = __import__("paper_2008_13145_amd")
    h, torch = gpu
    problems, X, Y = _mlp_data(n, k, k)
    p = synth.mlp_init(k)
    rng = np.random.default_rng(7)
    p["b1"] = rng.uniform(-0.1, 0.1, 64)
    p["b3"] = rng.uniform(-0.1, 0.1, k)
    P = _pack(p)
    p32 = _unpack(P, k)                      # oracle at exactly the FP32 weights
    X32 = X.astype(np.float32)
    g_ref, l_ref = omlp.grads(p32, X32.astype(np.float64), Y.astype(np.float32).astype(np.float64))
    dP = torch.from_numpy(P).cuda()
    dX = torch.from_numpy(X32).cuda()
    dY = torch.from_numpy(Y.astype(np.float32)).cuda()
    dG = torch.zeros_like(dP)
    dL = torch.zeros(1, dtype=torch.float32, device="cuda")
    dPred = torch.zeros((n, k), dtype=torch.float32, device="cuda")
    ws_bytes = kt_mod.Handle.mlp_workspace_bytes(n, 164, k)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    h.mlp_forward_backward(dP, dX, dY, n, k, dPred, dG, dL, ws, ws_bytes)
    torch.cuda.synchronize()
    g = _unpack(dG.cpu().numpy(), k)
    for name in omlp.PARAM_ORDER:
        ref = g_ref[name]
        err = np.linalg.norm(g[name] - ref) / max(np.linalg.norm(ref), 1e-30)
        assert err <= 1e-4, (name, err)
    assert abs(dL.item() / (n * k) - l_ref) <= 1e-4 * l_ref
    y_ref, _ = omlp.forward(p32, X32.astype(np.float64))
    assert np.max(np.abs(dPred.cpu().numpy() - y_ref)) <= 1e-4 * max(1.0, np.abs(y_ref).max())


def test_mlp_device_features(gpu):
    h, torch = gpu
    problems = synth.sweep_problems(50, 31)
    arr = np.array([[m, n, k, b, (ta | (tb << 32))] for (m, n, k, b, ta, tb) in problems], np.int64)
    dX = torch.zeros((len(problems), 6), dtype=torch.float32, device="cuda")
    h.mlp_features(torch.from_numpy(arr).cuda(), len(problems), dX)
    torch.cuda.synchronize()
    assert np.max(np.abs(dX.cpu().numpy() - omlp.features(problems))) <= 1e-6


def test_mlp_training_first_step_graph_and_selection(gpu):
    """One Adam step from given weights equals the closed form
    p - lr g / (|g| + eps); graph-replayed training equals step-by-step
    training bit for bit; batch selection is the argmax of the network."""
    kt_mod = __import__("paper_2008_13145_amd")
    h, torch = gpu
    k = 6
    problems = synth.sweep_problems(60, 4321)
    rng = np.random.default_rng(11)
    T = _planted_table(rng, len(problems), 30, 5)
    chosen = [1, 4, 9, 12, 20, 27]
    p0 = synth.mlp_init(k)
    P0 = _pack(p0)
    ws_bytes = kt_mod.Handle.mlp_workspace_bytes(len(problems), 30, k)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    h.fit_selector(3, problems, T, chosen, mlp_steps=1, mlp_init=P0, mlp_graph_steps=0,
                   workspace=ws, ws_bytes=ws_bytes)
    P1 = h.get_mlp()
    X = omlp.features(problems).astype(np.float32).astype(np.float64)
    Y = (onz.normalize(T, 0)[:, chosen] / 65535.0).astype(np.float32).astype(np.float64)
    g, _ = omlp.grads(_unpack(P0, k), X, Y)
    want = _pack({nm: _unpack(P0, k)[nm] - 1e-3 * g[nm] / (np.abs(g[nm]) + 1e-8)
                  for nm in omlp.PARAM_ORDER})
    # a coordinate whose gradient is tiny relative to eps may round differently
    gflat = _pack(g).astype(np.float64)
    sure = np.abs(gflat) > 1e-5
    assert np.allclose(P1[sure], want[sure], rtol=0, atol=2e-6)
    # graph replay vs eager: identical bits after 60 steps (and a second replay run)
    h.fit_selector(3, problems, T, chosen, mlp_steps=60, mlp_init=P0, mlp_graph_steps=0,
                   workspace=ws, ws_bytes=ws_bytes)
    eager = h.get_mlp()
    for _ in range(2):
        h.fit_selector(3, problems, T, chosen, mlp_steps=60, mlp_init=P0, mlp_graph_steps=20,
                       workspace=ws, ws_bytes=ws_bytes)
        assert np.array_equal(h.get_mlp(), eager)
    # batch selection == argmax of the FP64 forward at the trained FP32 weights
    arr = np.array([[m, n, kk, b, (ta | (tb << 32))] for (m, n, kk, b, ta, tb) in problems], np.int64)
    d_ids = torch.zeros(len(problems), dtype=torch.int32, device="cuda")
    h.select_batch(torch.from_numpy(arr).cuda(), len(problems), d_ids)
    torch.cuda.synchronize()
    y, _ = omlp.forward(_unpack(eager, k), omlp.features(problems))
    top2 = np.sort(y, axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > 1e-4
    ids = np.array(d_ids.cpu().tolist())
    want_ids = np.array([chosen[j] for j in np.argmax(y, axis=1)])
    assert np.array_equal(ids[clear], want_ids[clear])
    assert h.select(*problems[0]) == ids[0]


def test_exhaustive_selector_times_every_config_once_and_caches(gpu):
    """Exhaustive selection (the fallback and regret judge): the pick is a
    compiled configuration, is among the fastest of an independent sweep of
    the same shape, is cached, and the deployed path through it computes the
    product; device batch selection is refused for it."""
    import paper_2008_13145_amd as kt
    from oracle import gemm as og
    _, torch = gpu
    h = kt.Handle(0)
    try:
        h.fit_selector(kt.SEL_EXHAUSTIVE, [], np.zeros((0, 0), np.int64), [])
        s = (1024, 768, 512, 4, 1, 0)
        cid = h.select(*s)
        assert 0 <= cid < h.num_kernels()
        assert h.select(*s) == cid
        ws_bytes = kt.Handle.sweep_workspace_bytes([s])
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        T = h.sweep([s], ws, ws_bytes, target_ms=3.0)
        assert T[0, cid] <= 1.5 * T[0].min(), (cid, int(T[0, cid]), int(T[0].min()))
        M, N, K, bt, ta, tb = s
        a = synth.uniform_operand(synth.operand_seed(8, 0), bt * M * K).reshape(bt, M, K)
        b = synth.uniform_operand(synth.operand_seed(8, 1), bt * K * N).reshape(bt, K, N)
        dA = torch.from_numpy(np.ascontiguousarray(np.transpose(a, (0, 2, 1)))).cuda()
        dB = torch.from_numpy(b).cuda()
        dC = torch.full((bt, M, N), float("nan"), device="cuda")
        h.gemm(dA, dB, dC, ta, tb, 1.0, 0.0, config_id=-1)
        torch.cuda.synchronize()
        rows = np.arange(0, M, 97)
        cols = np.arange(0, N, 89)
        ref_r, ref_c = og.gemm_sampled(M, N, K, bt, 0, 0, 1.0, 0.0, a, K, M * K, b, N, K * N,
                                       None, N, M * N, rows, cols)
        C = dC.cpu().numpy()
        tol = 1e-5 * math.sqrt(K) * np.abs(a).max() * np.abs(b).max()
        assert np.all(np.abs(C[:, rows, :] - ref_r) <= tol)
        assert np.all(np.abs(C[:, :, cols] - ref_c) <= tol)
        h.fit_selector(kt.SEL_EXHAUSTIVE, [], np.zeros((0, 0), np.int64), [], dtype=kt.BF16)
        cb = h.select(*s, dtype=kt.BF16)
        assert 0 <= cb < h.num_kernels(kt.BF16)
        d_shapes = torch.zeros((1, 5), dtype=torch.int64, device="cuda")
        d_ids = torch.zeros(1, dtype=torch.int32, device="cuda")
        with pytest.raises(kt.KtError) as e:
            h.select_batch(d_shapes, 1, d_ids)
        assert e.value.status == -2
    finally:
        h.close()


@pytest.mark.parametrize("kind,n,d,k", [("random", 600, 16, 8), ("planted", 960, 12, 4),
                                        ("random", 97, 3, 5)])
def test_kmeans_u16_bitwise(gpu, kind, n, d, k):
    """k-means on arbitrary 16-bit vectors (the reduced-space pruning's
    clustering) equals the oracle bit for bit: labels, centroids, inertia."""
    kt_mod = __import__("paper_2008_13145_amd")
    h, torch = gpu
    rng = np.random.default_rng(n + d + k)
    if kind == "random":
        X = rng.integers(0, 65536, size=(n, d)).astype(np.uint16)
    else:
        centres = rng.integers(5000, 60000, size=(k, d))
        X = np.clip(centres[rng.integers(0, k, size=n)] + rng.integers(-2000, 2000, size=(n, d)),
                    0, 65535).astype(np.uint16)
    n_init, seed = 10, 13145
    ws_bytes = kt_mod.Handle.prune_workspace_bytes(n, d, k, n_init)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    got = h.kmeans_u16(X, k, seed, n_init, 300, workspace=ws, ws_bytes=ws_bytes)
    ref = okm.kmeans(X.astype(np.int64), k, _draws(seed, n_init, k), 300)
    assert got["inertia"] == ref["inertia"]
    assert np.array_equal(got["labels"], ref["labels"])
    assert np.array_equal(got["centroids"], ref["centroids"])


@pytest.mark.parametrize("norm", [0, 2])
def test_tree_pruning_on_gpu_normalized_table(gpu, norm):
    """Decision-tree pruning fed by the GPU normalization equals the oracle's
    normalization followed by the oracle's tree, pick for pick."""
    from oracle import prune_tree as opt
    from paper_2008_13145_amd import tune
    h, torch = gpu
    T, P, C, meta = tune.load_table(tune.DEFAULT_TABLE)
    train, _ = synth.train_test_split()
    rows = synth.rows_of_shapes(train)
    shapes = [tuple(int(v) for v in P[r]) for r in rows]
    got = tune.tree_pruning(h, T[rows], shapes, 8, norm)
    want = opt.prune(P[rows], onz.normalize(T[rows].astype(np.int64), norm), 8)
    assert got == want
