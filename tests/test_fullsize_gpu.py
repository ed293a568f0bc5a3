"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times: the sweep set's largest problems, each run through the deployed path
(k-means k = 8 on the measured table's training rows under the normalization
that scores best there, decision tree B fitted on them, kt_gemm with
config_id = -1), checked on sampled rows and columns of
sampled batch items against the FP64 oracle (the tolerance is per element,
so any subset is a valid check).

Operands are generated on the host (synth) exactly as stored in memory; the
transpose flags then define op(A) and op(B), so one buffer serves all four
layouts.
"""
import functools
import math
import os

import numpy as np
import pytest

import synth
from oracle import convert as cv
from oracle import gemm as og

pytestmark = pytest.mark.gpu

BIG = (3629, 3082, 3583, 28)          # the largest problem of the sweep set
WIDE = (2034, 3858, 470, 52)          # largest batch among the heavy problems
N_ROWS = 24                           # sampled rows / columns per checked item


def _table(dtype_name):
    from paper_2008_13145_amd import tune
    path = tune.table_path(dtype_name)
    if not os.path.exists(path):
        pytest.skip(f"no measured {dtype_name} table")
    T, P, C, meta = tune.load_table(path)
    return T, [tuple(int(v) for v in p) for p in P]


@pytest.fixture(scope="module")
def deployed(gpu):
    """A fresh handle with the deployed selectors of bench.py: per dtype,
    GPU k-means (k = 8, 10 restarts, normalization chosen on the training
    rows) on the training rows of its table and decision tree B over the
    chosen kernels."""
    import paper_2008_13145_amd as kt
    from paper_2008_13145_amd import tune
    _, torch = gpu
    h = kt.Handle(0)
    train, _ = synth.train_test_split()
    tr_rows = synth.rows_of_shapes(train)
    fitted = {}
    for name, dt in (("f32", kt.F32), ("bf16", kt.BF16), ("fp8", kt.FP8E4M3)):
        try:
            T, problems = _table(name)
        except pytest.skip.Exception:
            continue
        ws_bytes = kt.Handle.prune_workspace_bytes(len(tr_rows), T.shape[1], 8, 10)
        pws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        chosen = tune.select_pruning(h, T[tr_rows], 8, synth.SEED, workspace=pws,
                                     ws_bytes=ws_bytes)["chosen"]
        h.fit_selector(kt.SEL_DT_B, [problems[r] for r in tr_rows], T[tr_rows], chosen, dtype=dt)
        fitted[dt] = chosen
    torch.cuda.synchronize()
    return h, fitted


@functools.lru_cache(maxsize=2)
def _operands(M, N, K, bt):
    """Stored A (bt * M * K values) and B (bt * K * N values), flat; shared by
    the layouts and dtypes of one shape (no test writes them)."""
    a = synth.uniform_operand(synth.operand_seed(M, 0), bt * M * K)
    b = synth.uniform_operand(synth.operand_seed(M, 1), bt * K * N)
    return a, b


def _samples(M, N, bt, seed):
    rng = np.random.default_rng(seed)
    items = sorted(set([0, bt - 1] + list(rng.choice(bt, min(bt, 2), replace=False))))
    rows = np.sort(rng.choice(M, min(M, N_ROWS), replace=False))
    cols = np.sort(rng.choice(N, min(N, N_ROWS), replace=False))
    return items, rows, cols


def _oracle_item(a, b, M, N, K, ta, tb, i, rows, cols):
    """Sampled rows and columns of item i of op(A) op(B) in FP64."""
    lda = M if ta else K
    ldb = K if tb else N
    ai = a[i * M * K:(i + 1) * M * K]
    bi = b[i * K * N:(i + 1) * K * N]
    return og.gemm_sampled(M, N, K, 1, ta, tb, 1.0, 0.0, ai, lda, M * K, bi, ldb, K * N,
                           None, N, M * N, rows, cols)


@pytest.mark.parametrize("shape", [BIG, WIDE])
@pytest.mark.parametrize("ta,tb", synth.LAYOUTS)
def test_f32_deployed_path_full_size(deployed, gpu, shape, ta, tb):
    import paper_2008_13145_amd as kt
    h, fitted = deployed
    _, torch = gpu
    if kt.F32 not in fitted:
        pytest.skip("no FP32 table")
    M, N, K, bt = shape
    print(f"full-size FP32 {shape} layout {(ta, tb)} config {h.select(M, N, K, bt, ta, tb)}",
          flush=True)
    a, b = _operands(M, N, K, bt)
    dA = torch.from_numpy(a).cuda()
    dB = torch.from_numpy(b).cuda()
    dC = torch.full((bt * M * N,), float("nan"), dtype=torch.float32, device="cuda")
    h.gemm_raw(kt.F32, kt.shape(M, N, K, bt, ta, tb), 1.0, dA, M if ta else K, M * K,
               dB, K if tb else N, K * N, 0.0, dC, N, M * N, config_id=-1)
    torch.cuda.synchronize()
    items, rows, cols = _samples(M, N, bt, seed=K)
    C = dC.view(bt, M, N)
    for i in items:
        ref_r, ref_c = _oracle_item(a, b, M, N, K, ta, tb, i, rows, cols)
        ai = np.abs(a[i * M * K:(i + 1) * M * K]).max()
        bi = np.abs(b[i * K * N:(i + 1) * K * N]).max()
        tol = 1e-5 * math.sqrt(K) * ai * bi
        got_r = C[i][torch.from_numpy(rows).cuda(), :].cpu().numpy()
        got_c = C[i][:, torch.from_numpy(cols).cuda()].cpu().numpy()
        assert np.all(np.abs(got_r - ref_r[0]) <= tol), (i, float(np.abs(got_r - ref_r[0]).max()))
        assert np.all(np.abs(got_c - ref_c[0]) <= tol), (i, float(np.abs(got_c - ref_c[0]).max()))


@pytest.mark.parametrize("dtype_name", ["bf16", "fp8"])
@pytest.mark.parametrize("ta,tb", synth.LAYOUTS)
def test_lowp_deployed_path_full_size(deployed, gpu, dtype_name, ta, tb):
    """The largest problem through the deployed BF16 / FP8 path (conversion
    on the GPU from the same FP32 operands, as bench.py does): the relative
    Frobenius error of the sampled block against the FP64 oracle on the
    original FP32 values is within the stated bound (1e-2 BF16, 4e-2 FP8)."""
    import paper_2008_13145_amd as kt
    h, fitted = deployed
    _, torch = gpu
    dt = kt.BF16 if dtype_name == "bf16" else kt.FP8E4M3
    if dt not in fitted:
        pytest.skip(f"no {dtype_name} table")
    M, N, K, bt = BIG
    print(f"full-size {dtype_name} {BIG} layout {(ta, tb)} config "
          f"{h.select(M, N, K, bt, ta, tb, dtype=dt)}", flush=True)
    a, b = _operands(M, N, K, bt)
    d32a = torch.from_numpy(a).cuda()
    d32b = torch.from_numpy(b).cuda()
    eb = 2 if dt == kt.BF16 else 1
    dA = torch.empty(a.size * eb, dtype=torch.uint8, device="cuda")
    dB = torch.empty(b.size * eb, dtype=torch.uint8, device="cuda")
    scales = torch.empty(4, dtype=torch.float32, device="cuda")
    if dt == kt.BF16:
        h.convert_bf16(d32a, a.size, dA)
        h.convert_bf16(d32b, b.size, dB)
        sA = sB = None
    else:
        ws = torch.empty(16, dtype=torch.uint8, device="cuda")
        h.quantize_fp8(d32a, a.size, dA, scales[0:1], ws, 16)
        h.quantize_fp8(d32b, b.size, dB, scales[1:2], ws, 16)
        sA, sB = scales[0:1], scales[1:2]
    del d32a, d32b
    dC = torch.full((bt * M * N,), float("nan"), dtype=torch.float32, device="cuda")
    h.gemm_raw(dt, kt.shape(M, N, K, bt, ta, tb), 1.0, dA, M if ta else K, M * K,
               dB, K if tb else N, K * N, 0.0, dC, N, M * N, scaleA=sA, scaleB=sB,
               config_id=-1)
    torch.cuda.synchronize()
    bound = 1e-2 if dt == kt.BF16 else 4e-2
    items, rows, cols = _samples(M, N, bt, seed=K + 1)
    C = dC.view(bt, M, N)
    for i in items:
        ref_r, ref_c = _oracle_item(a, b, M, N, K, ta, tb, i, rows, cols)
        got_r = C[i][torch.from_numpy(rows).cuda(), :].cpu().numpy()
        got_c = C[i][:, torch.from_numpy(cols).cuda()].cpu().numpy()
        assert not np.isnan(got_r).any() and not np.isnan(got_c).any()
        e = math.hypot(cv.rel_frobenius(got_r, ref_r[0]) * np.linalg.norm(ref_r[0]),
                       cv.rel_frobenius(got_c, ref_c[0]) * np.linalg.norm(ref_c[0])) / \
            math.hypot(np.linalg.norm(ref_r[0]), np.linalg.norm(ref_c[0]))
        assert e <= bound, (i, e)
