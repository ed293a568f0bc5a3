"""GPU parity of the split-K GEMM (K cut into slices, FP32 partial planes,
one reduction pass) against the FP64 CPU oracle.

FP32: every element within the FP32 bound of the plain GEMM tests,
1e-5 * sqrt(K) * |alpha| * max|A_b| * max|B_b| + 2^-23 * |beta * C0|.
Small-integer operands make every partial sum exact, so the split-K result
must equal the oracle bit for bit whatever the slicing.  BF16 / FP8: the
same accuracy bars as the plain low-precision paths, against the oracle on
the dequantized operands."""
import math

import numpy as np
import pytest

import synth
from oracle import convert as cv
from oracle import gemm as og

pytestmark = pytest.mark.gpu

F32, BF16, FP8 = 0, 1, 2


def _stored(x, trans):
    return np.ascontiguousarray(np.transpose(x, (0, 2, 1)) if trans else x)


def _operands(M, N, K, bt, seed):
    a = synth.uniform_operand(synth.operand_seed(seed, 0), bt * M * K).reshape(bt, M, K)
    b = synth.uniform_operand(synth.operand_seed(seed, 1), bt * K * N).reshape(bt, K, N)
    c0 = synth.uniform_operand(synth.operand_seed(seed, 2), bt * M * N).reshape(bt, M, N)
    return a, b, c0


def _oracle(a, b, c0, alpha, beta):
    bt, M, K = a.shape
    N = b.shape[2]
    return og.gemm(M, N, K, bt, 0, 0, alpha, beta, a, K, M * K, b, N, K * N, c0, N, M * N)


def _bound(a, b, c0, alpha, beta):
    K = a.shape[2]
    amax = np.abs(a).reshape(a.shape[0], -1).max(axis=1)
    bmax = np.abs(b).reshape(b.shape[0], -1).max(axis=1)
    tol = 1e-5 * math.sqrt(max(K, 1)) * abs(alpha) * amax * bmax
    return tol[:, None, None] + 2.0 ** -23 * np.abs(beta * c0.astype(np.float64))


def _splitk(h, torch, dA, dB, c_init, ta, tb, splits, alpha, beta, cfg, dtype=F32, sA=None,
            sB=None):
    bt, M, N = c_init.shape
    K = dA.shape[1] if ta else dA.shape[2]
    ws_bytes = h.splitk_workspace_bytes(M, N, K, bt, splits)
    ws = torch.empty(max(ws_bytes, 4), dtype=torch.uint8, device="cuda")
    dC = torch.from_numpy(c_init.copy()).cuda()
    used = h.gemm_splitk(dA, dB, dC, splits, ws, ws_bytes, ta, tb, alpha, beta, config_id=cfg,
                         dtype=dtype, scaleA=sA, scaleB=sB)
    torch.cuda.synchronize()
    return dC.cpu().numpy(), used


def _expected_slices(K, splits):
    kc = -(-(-(-K // splits)) // 64) * 64
    return -(-K // kc)


@pytest.mark.parametrize("ta,tb", synth.LAYOUTS)
@pytest.mark.parametrize("M,N,K,bt,splits,beta", [
    (70, 45, 1000, 1, 4, 0.0),      # equal slices of 256 and a ragged 232-deep last one
    (37, 29, 777, 3, 5, 0.5),       # batched: one launch per slice; last slice 9 deep
    (130, 66, 4096, 1, 16, 0.0),    # 16 equal slices (one batched launch), 2 x 3 tiles
    (9, 300, 193, 2, 64, -1.0),     # more splits than 64-deep slices: S = 4
])
def test_splitk_fp32_parity(gpu, ta, tb, M, N, K, bt, splits, beta):
    h, torch = gpu
    a, b, c0 = _operands(M, N, K, bt, 700 + M)
    ref = _oracle(a, b, c0, 1.25, beta)
    dA = torch.from_numpy(_stored(a, ta)).cuda()
    dB = torch.from_numpy(_stored(b, tb)).cuda()
    init = c0 if beta != 0 else np.full_like(c0, np.nan)
    for cfg in (h.configs().index((32, 32, 2, 32)), h.configs().index((64, 64, 4, 16)),
                h.configs().index((16, 16, 1, 64))):
        got, used = _splitk(h, torch, dA, dB, init, ta, tb, splits, 1.25, beta, cfg)
        assert used == _expected_slices(K, splits)
        assert np.all(np.abs(got - ref) <= _bound(a, b, c0, 1.25, beta)), cfg


@pytest.mark.parametrize("splits", [2, 3, 7, 16])
def test_splitk_exact_integers(gpu, splits):
    """Integer operands in [-3, 3]: every partial plane and their sum are
    exact in FP32, so the result equals the oracle's bit for bit."""
    h, torch = gpu
    M, N, K, bt = 77, 131, 1500, 2
    rng = np.random.default_rng(splits)
    a = rng.integers(-3, 4, size=(bt, M, K)).astype(np.float32)
    b = rng.integers(-3, 4, size=(bt, K, N)).astype(np.float32)
    c0 = rng.integers(-5, 6, size=(bt, M, N)).astype(np.float32)
    ref = _oracle(a, b, c0, 2.0, -1.0)
    got, used = _splitk(h, torch, torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), c0, 0,
                        0, splits, 2.0, -1.0, h.configs().index((64, 64, 4, 16)))
    assert used == _expected_slices(K, splits)
    assert np.array_equal(got, ref.astype(np.float32))


def test_splitk_degenerate_cases(gpu):
    """One slice (splits 1, or K <= 64) is the plain GEMM, bit for bit and
    with no workspace; K = 0 gives beta * C; empty M is a no-op; a workspace
    smaller than the query is rejected before any launch."""
    import paper_2008_13145_amd as kt
    h, torch = gpu
    cfg = h.configs().index((32, 32, 2, 32))
    for (M, N, K, splits) in ((50, 40, 300, 1), (50, 40, 64, 8), (50, 40, 60, 3)):
        a, b, c0 = _operands(M, N, K, 1, 900 + K)
        dA, dB = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        assert h.splitk_workspace_bytes(M, N, K, 1, splits) == (0 if splits == 1 else
                                                               -(-splits * M * N * 4 // 256) * 256)
        got, used = _splitk(h, torch, dA, dB, c0, 0, 0, splits, 0.5, 2.0, cfg)
        assert used == 1
        dC = torch.from_numpy(c0.copy()).cuda()
        h.gemm(dA, dB, dC, 0, 0, 0.5, 2.0, config_id=cfg)
        torch.cuda.synchronize()
        assert np.array_equal(got, dC.cpu().numpy())
    # K = 0
    c0 = synth.uniform_operand(5, 6 * 7).reshape(1, 6, 7)
    dA = torch.zeros((1, 6, 0), dtype=torch.float32, device="cuda")
    dB = torch.zeros((1, 0, 7), dtype=torch.float32, device="cuda")
    got, used = _splitk(h, torch, dA, dB, c0, 0, 0, 4, 1.0, 3.0, cfg)
    assert np.array_equal(got, (np.float32(3.0) * c0).astype(np.float32))
    # empty M
    dA = torch.zeros((1, 0, 100), dtype=torch.float32, device="cuda")
    dB = torch.zeros((1, 100, 7), dtype=torch.float32, device="cuda")
    dC = torch.zeros((1, 0, 7), dtype=torch.float32, device="cuda")
    assert h.gemm_splitk(dA, dB, dC, 4, None, 0, config_id=cfg) == 1
    # too small a workspace
    a, b, c0 = _operands(40, 30, 500, 1, 3)
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    dC = torch.from_numpy(c0.copy()).cuda()
    with pytest.raises(kt.KtError) as e:
        h.gemm_splitk(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), dC, 4, ws, 256,
                      config_id=cfg)
    assert e.value.status == -5
    with pytest.raises(kt.KtError):
        h.gemm_splitk(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), dC, 65, ws, 256,
                      config_id=cfg)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), c0)


@pytest.mark.parametrize("dtype", [BF16, FP8])
@pytest.mark.parametrize("ta,tb", [(0, 1), (1, 0)])
def test_splitk_low_precision(gpu, dtype, ta, tb):
    """BF16 and FP8 slices: relative Frobenius error against the oracle on
    the original operands <= 1e-2 (BF16) / 4e-2 (FP8); against the
    dequantized operands BF16 within the FP32 bound, FP8 within 1e-3."""
    h, torch = gpu
    M, N, K, bt, splits = 96, 80, 2000, 1, 6
    a, b, c0 = _operands(M, N, K, bt, 1200 + dtype)
    As, Bs = _stored(a, ta), _stored(b, tb)
    dA32, dB32 = torch.from_numpy(As).cuda(), torch.from_numpy(Bs).cuda()
    sA = sB = None
    if dtype == BF16:
        dA = torch.zeros(As.shape, dtype=torch.int16, device="cuda")
        dB = torch.zeros(Bs.shape, dtype=torch.int16, device="cuda")
        h.convert_bf16(dA32, As.size, dA)
        h.convert_bf16(dB32, Bs.size, dB)
        qa = cv.bf16_decode(cv.bf16_rne(a)).astype(np.float64)
        qb = cv.bf16_decode(cv.bf16_rne(b)).astype(np.float64)
        cfg = h.configs(BF16).index((64, 64, 4, 64))
    else:
        dA = torch.zeros(As.shape, dtype=torch.uint8, device="cuda")
        dB = torch.zeros(Bs.shape, dtype=torch.uint8, device="cuda")
        sA = torch.zeros(1, dtype=torch.float32, device="cuda")
        sB = torch.zeros(1, dtype=torch.float32, device="cuda")
        w = torch.zeros(4, dtype=torch.int32, device="cuda")
        h.quantize_fp8(dA32, As.size, dA, sA, w, 16)
        h.quantize_fp8(dB32, Bs.size, dB, sB, w, 16)
        ca, fa = cv.quantize_fp8(a)
        cb, fb = cv.quantize_fp8(b)
        qa = cv.e4m3_decode(ca) / np.float64(fa)
        qb = cv.e4m3_decode(cb) / np.float64(fb)
        cfg = h.configs(FP8).index((64, 64, 4, 128))
    got, used = _splitk(h, torch, dA, dB, np.full_like(c0, np.nan), ta, tb, splits, 1.0, 0.0, cfg,
                        dtype=dtype, sA=sA, sB=sB)
    assert used == _expected_slices(K, splits)
    ref = _oracle(a, b, c0, 1.0, 0.0)
    ref_q = np.matmul(qa, qb)
    assert cv.rel_frobenius(got[0], ref[0]) <= (1e-2 if dtype == BF16 else 4e-2)
    if dtype == BF16:
        tol = 1e-5 * math.sqrt(K) * np.abs(qa).max() * np.abs(qb).max()
        assert np.all(np.abs(got - ref_q) <= tol)
    else:
        assert cv.rel_frobenius(got[0], ref_q[0]) <= 1e-3


def _auto_splits(tiles, K):
    S = 1
    while tiles * S < 2048 and S < 64 and K // (2 * S) >= 256:
        S *= 2
    return S


@pytest.mark.parametrize("M,N,K,bt", [(1, 4096, 25088, 1), (1, 1000, 4096, 1), (300, 200, 900, 2),
                                      (2000, 2000, 3000, 1)])
def test_splitk_automatic(gpu, M, N, K, bt):
    """splits = 0: S doubles while the configuration fills fewer than 2048
    work-groups and slices stay >= 256 deep (S < 64); results as in FP32
    parity."""
    h, torch = gpu
    cfg = h.configs().index((64, 64, 4, 16))
    a, b, c0 = _operands(M, N, K, bt, 40 + M)
    S = _auto_splits(-(-M // 64) * -(-N // 64) * bt, K)
    ref = _oracle(a, b, c0, 1.0, 0.0)
    got, used = _splitk(h, torch, torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(),
                        np.full_like(c0, np.nan), 0, 0, 0, 1.0, 0.0, cfg)
    assert used == _expected_slices(K, S)
    assert np.all(np.abs(got - ref) <= _bound(a, b, c0, 1.0, 0.0))
