"""The LDS-DMA pipeline of the BF16 / FP8 kernels (operands whose rows start
on 16-byte boundaries) against the register-staged pipeline and the oracle.

Both pipelines feed the same MFMAs with the same fragments in the same K
order, so on the same operands they must agree bit for bit, for every
configuration and layout, with ragged M and N, a partial last K stage, a
single partial stage and an empty K.  The register-staged run takes copies
of the operands placed 4 bytes off a 16-byte boundary, which routes it to
that pipeline (kt_dma_pipeline tells which one runs).  Every result is also
held to the accuracy bar against the FP64 oracle on the dequantized
operands: the FP32-accumulation bound for BF16 and a relative Frobenius
error of 1e-3 for FP8 (the FP8 MFMA does not accumulate at full FP32
precision)."""
import math

import numpy as np
import pytest

import synth
from oracle import convert as cv

pytestmark = pytest.mark.gpu

BF16, FP8 = 1, 2


def _stored(x, trans):
    return np.ascontiguousarray(np.transpose(x, (0, 2, 1)) if trans else x)


def _operand(h, torch, x, dtype):
    """Device copy of x (FP32 host array) in the low-precision format, its
    scale (FP8) and the dequantized values, plus a second copy 4 bytes off a
    16-byte boundary."""
    eb = 2 if dtype == BF16 else 1
    d32 = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    n = x.size
    q = torch.zeros(n * eb, dtype=torch.uint8, device="cuda")
    sc = torch.ones(1, dtype=torch.float32, device="cuda")
    if n == 0:
        deq = np.zeros(x.shape, np.float64)
    elif dtype == BF16:
        h.convert_bf16(d32, n, q)
        deq = cv.bf16_decode(cv.bf16_rne(x.astype(np.float32).ravel())).reshape(x.shape)
    else:
        amax = torch.zeros(4, dtype=torch.int32, device="cuda")
        h.quantize_fp8(d32, n, q, sc, amax, 16)
        codes, s = cv.quantize_fp8(x)
        deq = cv.e4m3_decode(codes) / np.float64(s)
    off = torch.zeros(n * eb + 32, dtype=torch.uint8, device="cuda")
    off[4:4 + n * eb] = q
    return q, off, sc, deq


def _run(h, torch, kt, dtype, shp, A, lda, sA, B, ldb, sB, scA, scB, cfg, c_init):
    dC = torch.from_numpy(c_init.copy()).cuda()
    bt, M, N = c_init.shape
    h.gemm_raw(dtype, shp, 1.25, A, lda, sA, B, ldb, sB, 0.5 if not np.isnan(c_init).any() else 0.0,
               dC, N, M * N, scaleA=scA.data_ptr(), scaleB=scB.data_ptr(), config_id=cfg)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


def _case(h, torch, kt, dtype, M, N, K, bt, ta, tb, cfgs, seed, beta=0.0):
    a = synth.uniform_operand(synth.operand_seed(seed, 0), bt * M * K).reshape(bt, M, K)
    b = synth.uniform_operand(synth.operand_seed(seed, 1), bt * K * N).reshape(bt, K, N)
    c0 = synth.uniform_operand(synth.operand_seed(seed, 2), bt * M * N).reshape(bt, M, N)
    qa, oa, sa, da = _operand(h, torch, _stored(a, ta), dtype)
    qb, ob, sb, db = _operand(h, torch, _stored(b, tb), dtype)
    deq_a = np.transpose(da, (0, 2, 1)) if ta else da
    deq_b = np.transpose(db, (0, 2, 1)) if tb else db
    ce = 8 if dtype == BF16 else 16      # an empty K keeps 16-byte rows
    lda, ldb = (M if ta else K) or ce, (K if tb else N) or ce
    shp = kt.shape(M, N, K, bt, ta, tb)
    assert h.dma_pipeline(dtype, shp, qa, lda, M * K, qb, ldb, K * N)
    assert not h.dma_pipeline(dtype, shp, oa.data_ptr() + 4, lda, M * K,
                                 ob.data_ptr() + 4, ldb, K * N)
    c_init = c0 if beta != 0 else np.full_like(c0, np.nan)
    ref = 1.25 * np.einsum("bik,bkj->bij", deq_a, deq_b)
    if beta != 0:
        ref = ref + beta * c0.astype(np.float64)
    amax = np.abs(deq_a).max() if deq_a.size else 0.0
    bmax = np.abs(deq_b).max() if deq_b.size else 0.0
    bad = []
    for cfg in cfgs:
        dma = _run(h, torch, kt, dtype, shp, qa, lda, M * K, qb, ldb, K * N, sa, sb, cfg, c_init)
        reg = _run(h, torch, kt, dtype, shp, oa.data_ptr() + 4, lda, M * K, ob.data_ptr() + 4,
                   ldb, K * N, sa, sb, cfg, c_init)
        if not np.array_equal(dma.view(np.uint32), reg.view(np.uint32)):
            bad.append((cfg, h.get_config(cfg, dtype), "differs from the register pipeline",
                        float(np.nanmax(np.abs(dma - reg)))))
            continue
        if dtype == BF16:
            tol = 1.25 * 1e-5 * math.sqrt(max(K, 1)) * amax * bmax + 2.0 ** -23 * abs(beta) * np.abs(c0)
            ok = bool(np.all(np.abs(dma - ref) <= tol))
        else:
            ok = all(cv.rel_frobenius(dma[i], ref[i]) <= 1e-3 for i in range(bt)) if K else \
                bool(np.all(np.abs(dma - ref) <= 2.0 ** -23 * abs(beta) * np.abs(c0)))
        if not ok:
            bad.append((cfg, h.get_config(cfg, dtype), "oracle", float(np.abs(dma - ref).max())))
    return bad


@pytest.mark.parametrize("dtype", [BF16, FP8])
@pytest.mark.parametrize("ta,tb", synth.LAYOUTS)
def test_every_config_both_pipelines(gpu, kt, dtype, ta, tb):
    """M, N ragged against every tile, K = 176 (a partial last stage for
    every K tile), two batch items."""
    h, torch = gpu
    M, N, K = (200, 144, 176) if dtype == BF16 else (208, 144, 176)
    bad = _case(h, torch, kt, dtype, M, N, K, 2, ta, tb, range(h.num_configs(dtype)),
                600 + 4 * dtype + 2 * ta + tb)
    assert not bad, bad[:6]


@pytest.mark.parametrize("dtype", [BF16, FP8])
@pytest.mark.parametrize("K", [0, 16, 64, 256, 1040])
def test_depths(gpu, kt, dtype, K):
    """Empty K (C = beta C), one partial stage, whole stages, several stages
    in flight with a tail; a spread of configurations, beta != 0."""
    h, torch = gpu
    n = h.num_configs(dtype)
    cfgs = sorted(set([0, 5, 29, 37, 48, 59, 66, 67, n - 1, n - 5, n - 13]))
    for ta, tb in synth.LAYOUTS:
        bad = _case(h, torch, kt, dtype, 96, 80, K, 1, ta, tb, cfgs, 700 + K + ta + 2 * tb,
                    beta=0.5)
        assert not bad, (ta, tb, bad[:4])


@pytest.mark.parametrize("dtype", [BF16, FP8])
def test_large_tiles_many_stages(gpu, kt, dtype):
    """The 256 x 256 and 128 x 128 tiles over a deep K on all layouts."""
    h, torch = gpu
    cfgs = [i for i, c in enumerate(h.configs(dtype)) if c[0] * c[1] >= 128 * 128]
    for ta, tb in synth.LAYOUTS:
        bad = _case(h, torch, kt, dtype, 512, 384, 1024, 1, ta, tb, cfgs, 800 + ta + 2 * tb)
        assert not bad, (ta, tb, bad[:4])


def _f32_dma_configs(h):
    """FP32 configurations with a DMA pipeline: t >= 2, whole-KiB tiles."""
    return [i for i, (bm, bn, t, bk) in enumerate(h.configs())
            if t >= 2 and (bm * bk * 4) % 1024 == 0 and (bn * bk * 4) % 1024 == 0]


@pytest.mark.parametrize("ta,tb", synth.LAYOUTS)
@pytest.mark.parametrize("M,N,K,bt,beta", [(200, 136, 172, 2, 0.0), (64, 96, 32, 1, -0.5),
                                           (132, 68, 1028, 1, 1.0)])
def test_f32_dma_every_config(gpu, kt, ta, tb, M, N, K, bt, beta):
    """FP32 through the DMA pipeline (16-byte rows, extents whole 4-float
    chunks; ragged against the tiles, a partial last K stage) on every
    configuration that has one, and the register-staged pipeline on operand
    copies 4 bytes off a 16-byte boundary: both within the FP32 bound
    1e-5 sqrt(K) |alpha| max|A| max|B| + 2^-23 |beta C0| of the oracle."""
    from oracle import gemm as og
    h, torch = gpu
    a = synth.uniform_operand(synth.operand_seed(950 + M, 0), bt * M * K).reshape(bt, M, K)
    b = synth.uniform_operand(synth.operand_seed(950 + N, 1), bt * K * N).reshape(bt, K, N)
    c0 = synth.uniform_operand(synth.operand_seed(950 + K, 2), bt * M * N).reshape(bt, M, N)
    ref = og.gemm(M, N, K, bt, 0, 0, 1.5, beta, a, K, M * K, b, N, K * N, c0, N, M * N)
    amax = np.abs(a).reshape(bt, -1).max(axis=1)
    bmax = np.abs(b).reshape(bt, -1).max(axis=1)
    tol = (1e-5 * math.sqrt(K) * 1.5 * amax * bmax)[:, None, None] + \
        2.0 ** -23 * np.abs(beta * c0.astype(np.float64))
    sa, sb = _stored(a, ta), _stored(b, tb)
    dA = torch.from_numpy(sa).cuda()
    dB = torch.from_numpy(sb).cuda()
    offA = torch.zeros(sa.size + 8, dtype=torch.float32, device="cuda")
    offB = torch.zeros(sb.size + 8, dtype=torch.float32, device="cuda")
    offA[1:1 + sa.size] = dA.reshape(-1)
    offB[1:1 + sb.size] = dB.reshape(-1)
    lda, ldb = (M if ta else K), (K if tb else N)
    shp = kt.shape(M, N, K, bt, ta, tb)
    assert h.dma_pipeline(kt.F32, shp, dA, lda, M * K, dB, ldb, K * N)
    assert not h.dma_pipeline(kt.F32, shp, offA.data_ptr() + 4, lda, M * K, offB.data_ptr() + 4,
                              ldb, K * N)
    init = c0 if beta != 0 else np.full_like(c0, np.nan)
    bad = []
    for cid in _f32_dma_configs(h):
        for (A, B) in ((dA, dB), (offA.data_ptr() + 4, offB.data_ptr() + 4)):
            dC = torch.from_numpy(init.copy()).cuda()
            h.gemm_raw(kt.F32, shp, 1.5, A, lda, M * K, B, ldb, K * N, beta, dC, N, M * N,
                       config_id=cid)
            torch.cuda.synchronize()
            got = dC.cpu().numpy()
            if not np.all(np.abs(got - ref) <= tol):
                bad.append((cid, h.get_config(cid), A is dA, float(np.nanmax(np.abs(got - ref)))))
    assert not bad, bad[:6]
