"""Split-K variants as selectable kernels (section 3's kernel type for deep
products with few output tiles): ids after the configurations, run by kt_gemm
with the handle's workspace, swept, pruned and selected like any kernel.

Parity: a variant forced through kt_gemm equals kt_gemm_splitk with the same
base configuration and slice count bit for bit (same kernels, same reduction
order), and both lie within the FP32 bound of the plain GEMM tests against
the FP64 oracle, 1e-5 * sqrt(K) * |alpha| * max|A_b| * max|B_b| +
2^-23 * |beta * C0|.  Without a workspace a variant is its base configuration
unsplit, bit for bit.  The selector's pick of a variant (kt_gemm(-1)) runs
that variant."""
import math

import numpy as np
import pytest

import synth
from oracle import gemm as og

pytestmark = pytest.mark.gpu

F32, BF16, FP8 = 0, 1, 2


def _operands(M, N, K, bt, seed):
    a = synth.uniform_operand(synth.operand_seed(seed, 0), bt * M * K).reshape(bt, M, K)
    b = synth.uniform_operand(synth.operand_seed(seed, 1), bt * K * N).reshape(bt, K, N)
    c0 = synth.uniform_operand(synth.operand_seed(seed, 2), bt * M * N).reshape(bt, M, N)
    return a, b, c0


def _stored(x, trans):
    return np.ascontiguousarray(np.transpose(x, (0, 2, 1)) if trans else x)


def _bound(a, b, c0, alpha, beta):
    K = a.shape[2]
    amax = np.abs(a).reshape(a.shape[0], -1).max(axis=1)
    bmax = np.abs(b).reshape(b.shape[0], -1).max(axis=1)
    tol = 1e-5 * math.sqrt(max(K, 1)) * abs(alpha) * amax * bmax
    return tol[:, None, None] + 2.0 ** -23 * np.abs(beta * c0.astype(np.float64))


def _variants(h, dtype=F32):
    n_cfg = h.num_configs(dtype)
    return [(v,) + h.get_kernel(v, dtype) for v in range(n_cfg, h.num_kernels(dtype))]


def test_kernel_ids_follow_the_configurations(gpu, kt):
    h, _ = gpu
    for dt in (F32, BF16, FP8):
        n_cfg = h.num_configs(dt)
        vs = _variants(h, dt)
        assert len(vs) == 24 and h.num_kernels(dt) == n_cfg + 24
        for v, (bm, bn, t, bk, sl), base in vs:
            assert 0 <= base < n_cfg and h.get_config(base, dt) == (bm, bn, t, bk)
            assert sl in (2, 4, 8, 16) and (bm == bn or {bm, bn} == {16, 128})
        for c in (0, n_cfg - 1):
            k, base = h.get_kernel(c, dt)
            assert base == c and k[4] == 1 and k[:4] == h.get_config(c, dt)


@pytest.mark.parametrize("ta,tb", synth.LAYOUTS)
@pytest.mark.parametrize("M,N,K,bt,beta", [(70, 45, 1000, 1, 0.0), (37, 29, 777, 3, 0.5),
                                           (130, 66, 4096, 1, -1.0)])
def test_forced_variant_equals_splitk(gpu, kt, ta, tb, M, N, K, bt, beta):
    h, torch = gpu
    a, b, c0 = _operands(M, N, K, bt, 900 + M + ta + 2 * tb)
    ref = og.gemm(M, N, K, bt, 0, 0, 1.5, beta, a, K, M * K, b, N, K * N, c0, N, M * N)
    tol = _bound(a, b, c0, 1.5, beta)
    dA = torch.from_numpy(_stored(a, ta)).cuda()
    dB = torch.from_numpy(_stored(b, tb)).cuda()
    init = c0 if beta != 0 else np.full_like(c0, np.nan)
    ws = torch.empty(kt.SPLIT_PLANE_CAP, dtype=torch.uint8, device="cuda")
    try:
        for v, (bm, bn, t, bk, sl), base in _variants(h):
            h.set_workspace(ws)
            dC = torch.from_numpy(init.copy()).cuda()
            h.gemm(dA, dB, dC, ta, tb, 1.5, beta, config_id=v)
            h.set_workspace(None)
            sk_bytes = kt.Handle.splitk_workspace_bytes(M, N, K, bt, sl)
            sws = torch.empty(max(sk_bytes, 4), dtype=torch.uint8, device="cuda")
            dS = torch.from_numpy(init.copy()).cuda()
            h.gemm_splitk(dA, dB, dS, sl, sws, sk_bytes, ta, tb, 1.5, beta, config_id=base)
            dP = torch.from_numpy(init.copy()).cuda()          # no workspace: the base, unsplit
            h.gemm(dA, dB, dP, ta, tb, 1.5, beta, config_id=v)
            dQ = torch.from_numpy(init.copy()).cuda()
            h.gemm(dA, dB, dQ, ta, tb, 1.5, beta, config_id=base)
            torch.cuda.synchronize()
            C, S, P, Q = (x.cpu().numpy() for x in (dC, dS, dP, dQ))
            assert np.array_equal(C.view(np.uint32), S.view(np.uint32)), (v, sl)
            assert np.array_equal(P.view(np.uint32), Q.view(np.uint32)), v
            assert np.all(np.abs(C - ref) <= tol), (v, float(np.abs(C - ref).max()))
    finally:
        h.set_workspace(None)


def test_workspace_query_and_cap(gpu, kt):
    h, _ = gpu
    v16 = next(v for v, k, _ in _variants(h) if k[4] == 16)
    assert h.kernel_workspace_bytes(64, 64, 4096, 1, id=v16) == 16 * 64 * 64 * 4
    assert h.kernel_workspace_bytes(64, 64, 100, 1, id=v16) == 2 * 64 * 64 * 4   # two 64-deep slices
    assert h.kernel_workspace_bytes(64, 64, 64, 1, id=v16) == 0                # one slice
    assert h.kernel_workspace_bytes(4096, 4096, 4096, 1, id=v16) == 0          # planes beyond the cap
    assert h.kernel_workspace_bytes(64, 64, 4096, 1, id=0) == 0                # a configuration


def test_selected_variant_runs_split(gpu, kt):
    """A table whose deep-K rows are fastest on one split-K variant: trees fit
    on it route kt_gemm(-1) to that variant, which matches the forced run bit
    for bit and the oracle within the bound."""
    h, torch = gpu
    hs = kt.Handle(0)
    try:
        n_k = hs.num_kernels()
        vs = _variants(hs)
        v = next(x for x, k, _ in vs if k[0] == 32 and k[4] == 8)
        plain = hs.get_config(0)
        problems = synth.sweep_problems(40, 4343)
        rng = np.random.default_rng(5)
        T = rng.integers(20000, 90000, size=(len(problems), n_k)).astype(np.int64)
        for i, p in enumerate(problems):
            T[i, v if p[2] >= 512 else 0] = 1000
        hs.fit_selector(kt.SEL_DT_A, problems, T, [0, v])
        hs.set_fallback(0)
        M, N, K, bt, ta, tb = 96, 80, 3000, 1, 0, 1
        assert hs.select(M, N, K, bt, ta, tb) == v
        assert hs.select(M, N, 100, bt, ta, tb) == 0
        a, b, c0 = _operands(M, N, K, bt, 77)
        ref = og.gemm(M, N, K, bt, 0, 0, 1.0, 0.0, a, K, M * K, b, N, K * N, None, N, M * N)
        dA = torch.from_numpy(a).cuda()
        dB = torch.from_numpy(_stored(b, 1)).cuda()
        ws = torch.empty(kt.SPLIT_PLANE_CAP, dtype=torch.uint8, device="cuda")
        hs.set_workspace(ws)
        dC = torch.full((bt, M, N), float("nan"), device="cuda")
        hs.gemm(dA, dB, dC, ta, tb, config_id=-1)
        dF = torch.full((bt, M, N), float("nan"), device="cuda")
        hs.gemm(dA, dB, dF, ta, tb, config_id=v)
        torch.cuda.synchronize()
        C, F = dC.cpu().numpy(), dF.cpu().numpy()
        assert np.array_equal(C.view(np.uint32), F.view(np.uint32))
        assert np.all(np.abs(C - ref) <= _bound(a, b, c0, 1.0, 0.0))
        assert plain == hs.get_kernel(0)[0][:4]
    finally:
        hs.close()


def test_sweep_times_variants(gpu, kt):
    h, torch = gpu
    problems = [(48, 40, 2048, 1, 0, 0), (130, 33, 700, 2, 1, 1)]
    vs = [v for v, _, _ in _variants(h)]
    ids = [0, 5] + vs[::3]
    ws_bytes = kt.Handle.sweep_workspace_bytes(problems)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    T = h.sweep(problems, ws, ws_bytes, config_ids=ids, target_ms=0.2, max_reps=20)
    assert (T > 0).all()
    # the operands alone do not leave room for the partial planes
    op_only = kt.Handle.sweep_workspace_bytes([(48, 40, 2048, 1, 0, 0)]) - \
        h.kernel_workspace_bytes(48, 40, 2048, 1, id=vs[3])
    with pytest.raises(kt.KtError) as e:
        h.sweep(problems[:1], ws, op_only, config_ids=[vs[3]], target_ms=0.2, max_reps=5)
    assert e.value.status == -5


def test_fallback_may_take_variants_of_chosen_configurations(gpu, kt):
    """Outside the training box the fallback times the chosen kernels and the
    split-K variants of their configurations; its pick is one of those and
    kt_gemm(-1) computes the product through it."""
    h, torch = gpu
    hs = kt.Handle(0)
    try:
        vs = _variants(hs)
        base16 = next(b for _, k, b in vs if k[0] == k[1] == 16)
        own = [v for v, k, b in vs if b == base16]
        problems = synth.sweep_problems(30, 4444)
        rng = np.random.default_rng(6)
        T = rng.integers(1000, 90000, size=(len(problems), hs.num_kernels())).astype(np.int64)
        chosen = [base16, hs.configs().index((64, 64, 4, 16))]
        hs.fit_selector(kt.SEL_DT_B, problems, T, chosen)
        M, N, K = 1, 512, 25088               # M = 1 lies below every training M
        pick = hs.select(M, N, K)
        assert pick in chosen + own
        a, b, c0 = _operands(M, N, K, 1, 91)
        ref = og.gemm(M, N, K, 1, 0, 0, 1.0, 0.0, a, K, M * K, b, N, K * N, None, N, M * N)
        ws = torch.empty(kt.SPLIT_PLANE_CAP, dtype=torch.uint8, device="cuda")
        hs.set_workspace(ws)
        dC = torch.full((1, M, N), float("nan"), device="cuda")
        hs.gemm(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), dC, config_id=-1)
        torch.cuda.synchronize()
        assert np.all(np.abs(dC.cpu().numpy() - ref) <= _bound(a, b, c0, 1.0, 0.0))
    finally:
        hs.close()


@pytest.mark.parametrize("dtype", [BF16, FP8])
def test_low_precision_variants_equal_splitk(gpu, kt, dtype):
    h, torch = gpu
    M, N, K, bt = 64, 96, 2048, 1
    a, b, _ = _operands(M, N, K, bt, 55 + dtype)
    dA32 = torch.from_numpy(a).cuda()
    dB32 = torch.from_numpy(_stored(b, 1)).cuda()
    eb = 2 if dtype == BF16 else 1
    dA = torch.empty(a.size * eb, dtype=torch.uint8, device="cuda")
    dB = torch.empty(b.size * eb, dtype=torch.uint8, device="cuda")
    sc = torch.ones(4, dtype=torch.float32, device="cuda")
    if dtype == BF16:
        h.convert_bf16(dA32, a.size, dA)
        h.convert_bf16(dB32, b.size, dB)
    else:
        amax = torch.empty(4, dtype=torch.float32, device="cuda")
        h.quantize_fp8(dA32, a.size, dA, sc[0:], amax, 16)
        h.quantize_fp8(dB32, b.size, dB, sc[1:], amax, 16)
    ws = torch.empty(kt.SPLIT_PLANE_CAP, dtype=torch.uint8, device="cuda")
    try:
        for v, (bm, bn, t, bk, sl), base in _variants(h, dtype):
            h.set_workspace(ws)
            dC = torch.zeros((bt, M, N), device="cuda")
            h.gemm_raw(dtype, kt.shape(M, N, K, bt, 0, 1), 1.0, dA, K, M * K, dB, K, N * K, 0.0,
                       dC, N, M * N, scaleA=sc[0:].data_ptr(), scaleB=sc[1:].data_ptr(),
                       config_id=v)
            h.set_workspace(None)
            sk = kt.Handle.splitk_workspace_bytes(M, N, K, bt, sl)
            sws = torch.empty(max(sk, 4), dtype=torch.uint8, device="cuda")
            dS = torch.zeros((bt, M, N), device="cuda")
            h.gemm_splitk_raw(dtype, kt.shape(M, N, K, bt, 0, 1), sl, 1.0, dA, K, M * K, dB, K,
                              N * K, 0.0, dS, N, M * N, sws, sk, scaleA=sc[0:].data_ptr(),
                              scaleB=sc[1:].data_ptr(), config_id=base)
            torch.cuda.synchronize()
            C, S = dC.cpu().numpy(), dS.cpu().numpy()
            assert np.array_equal(C.view(np.uint32), S.view(np.uint32)), (v, sl)
            ref = a[0].astype(np.float64) @ b[0].astype(np.float64)
            rel = np.linalg.norm(C[0] - ref) / np.linalg.norm(ref)
            assert rel <= (1e-2 if dtype == BF16 else 4e-2), (v, rel)
    finally:
        h.set_workspace(None)
