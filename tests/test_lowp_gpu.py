"""GPU parity of the BF16 and FP8-e4m3 paths against the CPU oracle.

Accuracy bar: relative Frobenius error per result (per batch item) against
the FP64 oracle on the original FP32 operands <= 1e-2 (BF16) and <= 4e-2
(FP8).  The kernel itself is checked tighter against the oracle on the
dequantized operands: BF16 within the FP32-accumulation bound; FP8 within a
relative Frobenius error of 1e-3, because gfx950's FP8 MFMA
(v_mfma_scale_f32_32x32x64_f8f6f4, unit block scales) does not accumulate at
full FP32 precision (measured: one instruction's error is about
2^-12 * sum |terms|), and every FP8 configuration built on the same MFMA
shape (16x16x128 for t = 2, 32x32x64 otherwise) must give the same bits.  BF16 is also checked bit for bit
where every value and partial sum is exact."""
import math

import numpy as np
import pytest

import synth
from oracle import convert as cv
from oracle import gemm as og

pytestmark = pytest.mark.gpu

BF16, FP8 = 1, 2


def _values(n, seed):
    x = synth.uniform_operand(seed, n).astype(np.float32)
    e = (synth.uniform_operand(seed + 1, n) * 24).astype(np.int32).astype(np.float32)
    return (x * np.float32(2.0) ** e).astype(np.float32)


def test_bf16_conversion_bitwise(gpu):
    h, torch = gpu
    x = np.concatenate([_values(1_000_003, 5),
                        np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 3.4e38, -3.4e38, 1e-40,
                                  1.00390625, 1.01171875], np.float32)])
    dx = torch.from_numpy(x).cuda()
    dy = torch.zeros(x.size, dtype=torch.int16, device="cuda")
    h.convert_bf16(dx, x.size, dy)
    torch.cuda.synchronize()
    assert np.array_equal(dy.cpu().numpy().view(np.uint16), cv.bf16_rne(x))


@pytest.mark.parametrize("scale_exp", [0, -20, 12])
def test_fp8_quantization_bitwise(gpu, scale_exp):
    h, torch = gpu
    x = (synth.uniform_operand(7 + scale_exp, 1_000_001) * np.float32(2.0 ** scale_exp)).astype(np.float32)
    x[::1000] = 0.0
    x[5] = -x[5]
    dx = torch.from_numpy(x).cuda()
    dy = torch.zeros(x.size, dtype=torch.uint8, device="cuda")
    ds = torch.zeros(1, dtype=torch.float32, device="cuda")
    ws = torch.zeros(4, dtype=torch.int32, device="cuda")
    h.quantize_fp8(dx, x.size, dy, ds, ws, 16)
    torch.cuda.synchronize()
    codes, s = cv.quantize_fp8(x)
    assert ds.item() == float(s)
    assert np.array_equal(dy.cpu().numpy(), codes)


def test_fp8_quantization_zero_and_empty(gpu):
    h, torch = gpu
    dx = torch.zeros(100, dtype=torch.float32, device="cuda")
    dy = torch.full((100,), 7, dtype=torch.uint8, device="cuda")
    ds = torch.zeros(1, dtype=torch.float32, device="cuda")
    ws = torch.zeros(4, dtype=torch.int32, device="cuda")
    h.quantize_fp8(dx, 100, dy, ds, ws, 16)
    torch.cuda.synchronize()
    assert ds.item() == 1.0 and not dy.cpu().numpy().any()
    h.quantize_fp8(dx, 0, dy, ds, ws, 16)
    torch.cuda.synchronize()
    assert ds.item() == 1.0


def _stored(a_op, trans):
    return np.ascontiguousarray(np.transpose(a_op, (0, 2, 1)) if trans else a_op)


def _prepare(h, torch, a, b, ta, tb, dtype):
    """Device operands of dtype from FP32 op() matrices; returns tensors, the
    dequantized op() matrices (float64) and the scale tensors."""
    As, Bs = _stored(a, ta), _stored(b, tb)
    dA32 = torch.from_numpy(As).cuda()
    dB32 = torch.from_numpy(Bs).cuda()
    if dtype == BF16:
        dA = torch.zeros(As.shape, dtype=torch.int16, device="cuda")
        dB = torch.zeros(Bs.shape, dtype=torch.int16, device="cuda")
        h.convert_bf16(dA32, As.size, dA)
        h.convert_bf16(dB32, Bs.size, dB)
        deq_a = cv.bf16_decode(cv.bf16_rne(a)).astype(np.float64)
        deq_b = cv.bf16_decode(cv.bf16_rne(b)).astype(np.float64)
        return dA, dB, None, None, deq_a, deq_b
    dA = torch.zeros(As.shape, dtype=torch.uint8, device="cuda")
    dB = torch.zeros(Bs.shape, dtype=torch.uint8, device="cuda")
    sA = torch.zeros(1, dtype=torch.float32, device="cuda")
    sB = torch.zeros(1, dtype=torch.float32, device="cuda")
    ws = torch.zeros(4, dtype=torch.int32, device="cuda")
    h.quantize_fp8(dA32, As.size, dA, sA, ws, 16)
    h.quantize_fp8(dB32, Bs.size, dB, sB, ws, 16)
    qa, sa = cv.quantize_fp8(a)
    qb, sb = cv.quantize_fp8(b)
    deq_a = cv.e4m3_decode(qa) / np.float64(sa)
    deq_b = cv.e4m3_decode(qb) / np.float64(sb)
    return dA, dB, sA, sB, deq_a, deq_b


def _gemm(h, torch, dtype, dA, dB, sA, sB, shape, ta, tb, alpha, beta, c0, cfg):
    import paper_2008_13145_amd as kt
    bt, M, N = c0.shape
    K = shape
    dC = torch.from_numpy(c0.copy()).cuda()
    lda = M if ta else K
    ldb = K if tb else N
    h.gemm_raw(dtype, kt.shape(M, N, K, bt, ta, tb), alpha, dA, lda, M * K, dB, ldb, K * N, beta,
               dC, N, M * N, scaleA=sA, scaleB=sB, config_id=cfg)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


def _ref(a, b, c0, alpha, beta):
    bt, M, K = a.shape
    N = b.shape[2]
    return og.gemm(M, N, K, bt, 0, 0, alpha, beta, a.astype(np.float32), K, M * K,
                   b.astype(np.float32), N, K * N, c0, N, M * N)


def _ref64(a, b, c0, alpha, beta):
    # exact-input reference for dequantized operands (not representable in FP32 for FP8)
    out = alpha * np.einsum("bik,bkj->bij", a, b)
    if beta != 0:
        out = out + beta * c0.astype(np.float64)
    return out


@pytest.mark.parametrize("dtype", [BF16, FP8])
@pytest.mark.parametrize("ta,tb", synth.LAYOUTS)
def test_all_configs_accuracy(gpu, dtype, ta, tb):
    h, torch = gpu
    M, N, K, bt = 300, 270, 200, 2
    a = synth.uniform_operand(synth.operand_seed(50 + ta, 0), bt * M * K).reshape(bt, M, K)
    b = synth.uniform_operand(synth.operand_seed(50 + tb, 1), bt * K * N).reshape(bt, K, N)
    c0 = synth.uniform_operand(synth.operand_seed(52, 2), bt * M * N).reshape(bt, M, N)
    dA, dB, sA, sB, deq_a, deq_b = _prepare(h, torch, a, b, ta, tb, dtype)
    alpha, beta = 1.0, 0.0
    ref = _ref(a, b, c0, alpha, beta)
    ref_q = _ref64(deq_a, deq_b, c0, alpha, beta)
    bound = 1e-2 if dtype == BF16 else 4e-2
    tol_q = 1e-5 * math.sqrt(K) * np.abs(deq_a).max() * np.abs(deq_b).max()
    bad = []
    first = {}          # per MFMA shape: 16x16 blocks (t = 2) or 32x32 blocks
    for cfg in range(h.num_configs(dtype)):
        got = _gemm(h, torch, dtype, dA, dB, sA, sB, K, ta, tb, alpha, beta,
                    np.full_like(c0, np.nan), cfg)
        fam = first.setdefault(h.get_config(cfg, dtype)[2] == 2, got)
        for i in range(bt):
            e = cv.rel_frobenius(got[i], ref[i])
            if dtype == BF16:
                tight = bool(np.all(np.abs(got[i] - ref_q[i]) <= tol_q))
            else:
                tight = cv.rel_frobenius(got[i], ref_q[i]) <= 1e-3 and np.array_equal(got, fam)
            if not e <= bound or not tight:
                bad.append((cfg, h.get_config(cfg, dtype), e))
    assert not bad, bad[:8]


@pytest.mark.parametrize("ta,tb", synth.LAYOUTS)
def test_all_configs_exact_integers_bf16(gpu, ta, tb):
    """Integers in [-7, 7] are exact in BF16 and every partial sum is an
    integer below 2^24, so every configuration equals the oracle bit for bit."""
    h, torch = gpu
    M, N, K, bt = 133, 96, 160, 2
    rng = np.random.default_rng(ta * 2 + tb)
    a = rng.integers(-7, 8, size=(bt, M, K)).astype(np.float32)
    b = rng.integers(-7, 8, size=(bt, K, N)).astype(np.float32)
    c0 = np.zeros((bt, M, N), np.float32)
    dA, dB, sA, sB, _, _ = _prepare(h, torch, a, b, ta, tb, BF16)
    ref = _ref(a, b, c0, 1.0, 0.0)
    bad = []
    for cfg in range(h.num_configs(BF16)):
        got = _gemm(h, torch, BF16, dA, dB, sA, sB, K, ta, tb, 1.0, 0.0, np.full_like(c0, np.nan), cfg)
        if not np.array_equal(got.astype(np.float64), ref):
            bad.append((cfg, h.get_config(cfg, BF16)))
    assert not bad, bad[:8]


@pytest.mark.parametrize("ta,tb", synth.LAYOUTS)
def test_fp8_one_mfma_block_exact(gpu, ta, tb):
    """FP8 with K = 16 (inside one 64-deep MFMA) and values k * 64, k in
    [-7, 7] (exact e4m3 codes after the power-of-two scale 448 / 7 = 64): the
    sum is exact, so every configuration equals the oracle."""
    h, torch = gpu
    M, N, K, bt = 70, 45, 16, 1
    rng = np.random.default_rng(10 + ta * 2 + tb)
    a = rng.integers(-7, 8, size=(bt, M, K)).astype(np.float32)
    b = rng.integers(-7, 8, size=(bt, K, N)).astype(np.float32)
    a[:, 0, 0] = 7
    b[:, 0, 0] = -7
    c0 = np.zeros((bt, M, N), np.float32)
    dA, dB, sA, sB, _, _ = _prepare(h, torch, a, b, ta, tb, FP8)
    ref = _ref(a, b, c0, 1.0, 0.0)
    bad = []
    for cfg in range(h.num_configs(FP8)):
        got = _gemm(h, torch, FP8, dA, dB, sA, sB, K, ta, tb, 1.0, 0.0, np.full_like(c0, np.nan), cfg)
        if not np.array_equal(got.astype(np.float64), ref):
            bad.append((cfg, h.get_config(cfg, FP8), float(np.abs(got - ref).max())))
    assert not bad, bad[:8]


@pytest.mark.parametrize("dtype", [BF16, FP8])
def test_edge_shapes_alpha_beta(gpu, dtype):
    h, torch = gpu
    cfgs = h.configs(dtype)
    picks = [0, len(cfgs) // 3, len(cfgs) // 2, len(cfgs) - 1]
    for (M, N, K, bt) in [(1, 1, 1, 1), (17, 31, 13, 1), (255, 257, 129, 1), (33, 1, 300, 3)]:
        for (ta, tb) in synth.LAYOUTS:
            a = synth.uniform_operand(M * 7 + ta, bt * M * K).reshape(bt, M, K)
            b = synth.uniform_operand(N * 5 + tb, bt * K * N).reshape(bt, K, N)
            c0 = synth.uniform_operand(99, bt * M * N).reshape(bt, M, N)
            dA, dB, sA, sB, deq_a, deq_b = _prepare(h, torch, a, b, ta, tb, dtype)
            for alpha, beta in ((1.0, 0.0), (-0.5, 2.0)):
                ref_q = _ref64(deq_a, deq_b, c0, alpha, beta)
                # BF16: FP32-accumulation bound; FP8: the MFMA's ~12-bit accumulation
                acc_rel = 1e-5 * math.sqrt(K) if dtype == BF16 else 2.0 ** -14 * K
                tol = acc_rel * abs(alpha) * np.abs(deq_a).max() * np.abs(deq_b).max() \
                    + 2.0 ** -23 * np.abs(beta * c0)
                for cfg in picks:
                    c_init = np.full_like(c0, np.nan) if beta == 0 else c0
                    got = _gemm(h, torch, dtype, dA, dB, sA, sB, K, ta, tb, alpha, beta, c_init, cfg)
                    assert not np.isnan(got).any()
                    assert np.all(np.abs(got - ref_q) <= tol), (M, N, K, bt, ta, tb, alpha, cfgs[cfg])


@pytest.mark.parametrize("dtype", [BF16, FP8])
@pytest.mark.parametrize("ta,tb", synth.LAYOUTS)
def test_unaligned_rows_and_bases(gpu, dtype, ta, tb):
    """Leading dimensions that leave rows off 4-byte boundaries take the
    realigned-window loads; a base pointer off a 4-byte boundary takes the
    element loads.  Both must match the dense reference."""
    import paper_2008_13145_amd as kt
    h, torch = gpu
    M, N, K = 75, 61, 53
    a = synth.uniform_operand(3 + ta, M * K).reshape(1, M, K)
    b = synth.uniform_operand(4 + tb, K * N).reshape(1, K, N)
    _, _, sA, sB, deq_a, deq_b = _prepare(h, torch, a, b, ta, tb, dtype)
    qa = cv.bf16_rne(a) if dtype == BF16 else cv.quantize_fp8(a)[0]
    qb = cv.bf16_rne(b) if dtype == BF16 else cv.quantize_fp8(b)[0]
    As, Bs = _stored(qa, ta)[0], _stored(qb, tb)[0]
    ref_q = _ref64(deq_a, deq_b, np.zeros((1, M, N), np.float32), 1.0, 0.0)[0]
    acc_rel = 1e-5 * math.sqrt(K) if dtype == BF16 else 2.0 ** -14 * K
    tol = acc_rel * np.abs(deq_a).max() * np.abs(deq_b).max()
    tdt = torch.int16 if dtype == BF16 else torch.uint8
    eb = 2 if dtype == BF16 else 1
    cfgs = h.configs(dtype)
    for pad_a, pad_b, off in ((1, 3, 0), (0, 0, 1), (5, 2, 2)):
        lda, ldb = As.shape[1] + pad_a, Bs.shape[1] + pad_b
        bufA = torch.zeros(off + As.shape[0] * lda + 8, dtype=tdt, device="cuda")
        bufB = torch.zeros(off + Bs.shape[0] * ldb + 8, dtype=tdt, device="cuda")
        bufA[off:off + As.shape[0] * lda].view(As.shape[0], lda)[:, :As.shape[1]] = \
            torch.from_numpy(As.view(np.int16) if dtype == BF16 else As).cuda()
        bufB[off:off + Bs.shape[0] * ldb].view(Bs.shape[0], ldb)[:, :Bs.shape[1]] = \
            torch.from_numpy(Bs.view(np.int16) if dtype == BF16 else Bs).cuda()
        for cfg in (0, 17, 40, len(cfgs) - 1):
            dC = torch.zeros((M, N), dtype=torch.float32, device="cuda")
            h.gemm_raw(dtype, kt.shape(M, N, K, 1, ta, tb), 1.0, bufA.data_ptr() + off * eb, lda, 0,
                       bufB.data_ptr() + off * eb, ldb, 0, 0.0, dC, N, 0, scaleA=sA, scaleB=sB,
                       config_id=cfg)
            torch.cuda.synchronize()
            assert np.all(np.abs(dC.cpu().numpy() - ref_q) <= tol), (pad_a, pad_b, off, cfgs[cfg])


def test_lowp_sweep(gpu):
    import paper_2008_13145_amd as kt
    h, torch = gpu
    problems = [(256, 256, 256, 1, 0, 1), (100, 60, 70, 3, 1, 0)]
    for dtype in (BF16, FP8):
        ws_bytes = kt.Handle.sweep_workspace_bytes(problems, dtype)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        T = h.sweep(problems, ws, ws_bytes, config_ids=[0, 10, 30, 58], target_ms=0.2,
                    max_reps=10, dtype=dtype)
        assert (T > 0).all()


@pytest.mark.parametrize("cfg_t,K", [(4, 64), (2, 128)])
def test_fp8_mfma_accumulation_error_measured(gpu, cfg_t, K):
    """The evidence behind the FP8 bounds: one K step of exactly one MFMA
    (64 deep for the 32x32 blocks, 128 for the 16x16 ones) on random e4m3
    codes with unit scales, against the exact sum of the products (every
    product and partial sum is exact in FP64).  The error per element stays
    within 2^-11 of the sum of the magnitudes of its terms (the accumulation
    inside the instruction is not full FP32; measured about 2^-12), which
    over K / depth instructions gives the K-linear bound the tests use."""
    import paper_2008_13145_amd as kt
    h, torch = gpu
    M = N = 64
    rng = np.random.default_rng(31 + K)
    codes_a = rng.integers(0, 256, size=(M, K)).astype(np.uint8)
    codes_b = rng.integers(0, 256, size=(N, K)).astype(np.uint8)
    for c in (codes_a, codes_b):
        c[(c & 0x7F) == 0x7F] = 0x38          # no NaN codes (0x38 = 1.0)
    a = cv.e4m3_decode(codes_a).astype(np.float64)
    b = cv.e4m3_decode(codes_b).astype(np.float64)
    exact = a @ b.T
    mag = np.abs(a) @ np.abs(b).T
    dA = torch.from_numpy(codes_a).cuda()
    dB = torch.from_numpy(codes_b).cuda()
    sc = torch.ones(2, dtype=torch.float32, device="cuda")
    cfgs = h.configs(FP8)
    cid = next(i for i, c in enumerate(cfgs) if c[2] == cfg_t and c[3] == K and c[0] == c[1] == 64)
    dC = torch.full((M, N), float("nan"), device="cuda")
    h.gemm_raw(FP8, kt.shape(M, N, K, 1, 0, 1), 1.0, dA, K, 0, dB, K, 0, 0.0, dC, N, 0,
               scaleA=sc[0:].data_ptr(), scaleB=sc[1:].data_ptr(), config_id=cid)
    torch.cuda.synchronize()
    got = dC.cpu().numpy().astype(np.float64)
    ratio = np.abs(got - exact) / np.maximum(mag, 1e-300)
    assert ratio.max() <= 2.0 ** -11, float(np.log2(ratio.max()))
