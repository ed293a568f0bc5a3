"""GPU parity of the FP32 GEMM family against the FP64 CPU oracle.

Tolerance (per element, FP32): |C_gpu - C*| <= 1e-5 * sqrt(K) * |alpha| *
max|A_b| * max|B_b| + 2^-23 * |beta * C0| -- the stated FP32 bound with
max-abs norms per batch item.  Identity and small-integer operands, whose
every partial sum is exact in FP32, must match bit for bit in all 656
instantiations (this also exposes LDS races: every configuration and
layout must produce the same bits).
"""
import math

import numpy as np
import pytest

import synth
from oracle import gemm as og

pytestmark = pytest.mark.gpu


def _stored(a_op, trans):
    """Row-major storage (batch, rows, cols) of op() matrices for a transpose flag."""
    return np.ascontiguousarray(np.transpose(a_op, (0, 2, 1)) if trans else a_op)


def _problem(M, N, K, bt, ta, tb, seed, beta=0.0):
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
    amax = np.abs(a).reshape(a.shape[0], -1).max(axis=1) if a.size else np.zeros(a.shape[0])
    bmax = np.abs(b).reshape(b.shape[0], -1).max(axis=1) if b.size else np.zeros(b.shape[0])
    tol = 1e-5 * math.sqrt(max(K, 1)) * abs(alpha) * amax * bmax
    return tol[:, None, None] + 2.0 ** -23 * np.abs(beta * c0.astype(np.float64))


def _run(h, torch, a, b, c0, ta, tb, alpha, beta, cfg, c_init=None):
    dA = torch.from_numpy(_stored(a, ta)).cuda()
    dB = torch.from_numpy(_stored(b, tb)).cuda()
    dC = torch.from_numpy(c0.copy() if c_init is None else c_init.copy()).cuda()
    h.gemm(dA, dB, dC, ta, tb, alpha, beta, config_id=cfg)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


def test_fill_matches_host_generator(gpu):
    h, torch = gpu
    for seed, n, off in ((1, 1000, 0), (synth.operand_seed(9, 1), 123457, 77), (2 ** 64 - 5, 4099, 3)):
        d = torch.empty(n, dtype=torch.float32, device="cuda")
        h.fill_uniform(d, n, seed, off)
        torch.cuda.synchronize()
        assert np.array_equal(d.cpu().numpy(), synth.uniform_operand(seed, n, offset=off))


def test_single_gemm_256_config_64x64x4x16(gpu):
    """The single-GEMM workload: 256^3, NN, alpha 1, beta 0, config (64,64,T4,BK16)."""
    h, torch = gpu
    cfg = h.configs().index((64, 64, 4, 16))
    a, b, c0 = _problem(256, 256, 256, 1, 0, 0, synth.SEED + 1)
    got = _run(h, torch, a, b, np.full_like(c0, np.nan), 0, 0, 1.0, 0.0, cfg)
    ref = _oracle(a, b, c0, 1.0, 0.0)
    assert np.all(np.abs(got - ref) <= _bound(a, b, c0, 1.0, 0.0))


@pytest.mark.parametrize("ta,tb", synth.LAYOUTS)
def test_all_configs_random_ragged(gpu, ta, tb):
    """Every configuration on a shape that spans several tiles with ragged
    M, N and K tails in every configuration (300 = 2*128+44, 100 = 64+36)."""
    h, torch = gpu
    M, N, K, bt = 300, 270, 100, 2
    a, b, c0 = _problem(M, N, K, bt, ta, tb, 1000 + 2 * ta + tb)
    alpha, beta = 0.75, -1.5
    ref = _oracle(a, b, c0, alpha, beta)
    tol = _bound(a, b, c0, alpha, beta)
    dA = torch.from_numpy(_stored(a, ta)).cuda()
    dB = torch.from_numpy(_stored(b, tb)).cuda()
    bad = []
    for cfg in range(h.num_configs()):
        dC = torch.from_numpy(c0.copy()).cuda()
        h.gemm(dA, dB, dC, ta, tb, alpha, beta, config_id=cfg)
        got = dC.cpu().numpy()
        err = np.abs(got - ref)
        if not np.all(err <= tol):
            bad.append((cfg, h.get_config(cfg), float(err.max()), float(tol.min())))
    assert not bad, bad[:10]


@pytest.mark.parametrize("ta,tb", synth.LAYOUTS)
def test_all_configs_exact_integer_operands(gpu, ta, tb):
    """Small-integer operands: every partial sum is an integer below 2^24, so
    every summation order is exact and all configurations equal the oracle
    bit for bit."""
    h, torch = gpu
    M, N, K, bt = 133, 70, 150, 2
    i = np.arange(M)[:, None]
    k = np.arange(K)[None, :]
    a = np.stack([((i + k + s) % 5 - 2) for s in range(bt)]).astype(np.float32)
    kk = np.arange(K)[:, None]
    j = np.arange(N)[None, :]
    b = np.stack([((j + 2 * kk + s) % 7 - 3) for s in range(bt)]).astype(np.float32)
    c0 = np.zeros((bt, M, N), np.float32)
    ref = _oracle(a, b, c0, 1.0, 0.0)
    assert np.abs(ref).max() < 2 ** 24
    dA = torch.from_numpy(_stored(a, ta)).cuda()
    dB = torch.from_numpy(_stored(b, tb)).cuda()
    bad = []
    for cfg in range(h.num_configs()):
        dC = torch.full((bt, M, N), float("nan"), dtype=torch.float32, device="cuda")
        h.gemm(dA, dB, dC, ta, tb, 1.0, 0.0, config_id=cfg)
        got = dC.cpu().numpy().astype(np.float64)
        if not np.array_equal(got, ref):
            bad.append((cfg, h.get_config(cfg)))
    assert not bad, bad[:10]


@pytest.mark.parametrize("ta,tb", synth.LAYOUTS)
def test_identity_bitwise(gpu, ta, tb):
    h, torch = gpu
    M = K = 129
    N = 77
    a = np.eye(M, dtype=np.float32)[None]
    b = synth.uniform_operand(3, K * N).reshape(1, K, N)
    for cfg in range(0, h.num_configs(), 3):
        got = _run(h, torch, a, b, np.full((1, M, N), np.nan, np.float32), ta, tb, 1.0, 0.0, cfg)
        assert np.array_equal(got, b), cfg


EDGE_SHAPES = [(1, 1, 1, 1), (17, 31, 13, 1), (255, 256, 257, 1), (256, 255, 1, 3),
               (257, 1, 64, 2), (1, 257, 33, 1), (64, 64, 1, 1), (9, 130, 200, 3)]


@pytest.mark.parametrize("M,N,K,bt", EDGE_SHAPES)
def test_edge_shapes_alpha_beta(gpu, M, N, K, bt):
    h, torch = gpu
    cfgs = h.configs()
    # one configuration of every thread tile and K tile, both small and large tiles
    picks = [cfgs.index(c) for c in [(8, 8, 1, 8), (16, 64, 1, 64), (32, 16, 2, 16),
                                       (128, 32, 2, 32), (32, 32, 4, 8), (128, 128, 4, 64),
                                       (64, 128, 8, 16), (128, 128, 8, 64)]]
    for (ta, tb) in synth.LAYOUTS:
        a, b, c0 = _problem(M, N, K, bt, ta, tb, 7 * M + N + K + bt)
        for alpha, beta in ((1.0, 0.0), (-0.5, 2.0), (2.0, 1.0), (0.0, -0.5)):
            ref = _oracle(a, b, c0, alpha, beta)
            tol = _bound(a, b, c0, alpha, beta)
            c_init = np.full_like(c0, np.nan) if beta == 0.0 else c0
            for cfg in picks:
                got = _run(h, torch, a, b, c0, ta, tb, alpha, beta, cfg, c_init=c_init)
                assert not np.isnan(got).any()
                assert np.all(np.abs(got - ref) <= tol), (ta, tb, alpha, beta, cfgs[cfg])


def test_k_zero_and_empty(gpu):
    h, torch = gpu
    c0 = synth.uniform_operand(5, 3 * 4 * 5).reshape(3, 4, 5)
    dC = torch.from_numpy(c0.copy()).cuda()
    dA = torch.zeros((3, 4, 0), dtype=torch.float32, device="cuda")
    dB = torch.zeros((3, 0, 5), dtype=torch.float32, device="cuda")
    h.gemm_raw(0, h_shape(0, 4, 5, 0, 3), 1.0, dA, 1, 0, dB, 5, 0, -0.5, dC, 5, 20, config_id=10)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), np.float32(-0.5) * c0)
    # M = 0: no-op, C untouched
    dC2 = torch.from_numpy(c0.copy()).cuda()
    h.gemm_raw(0, h_shape(0, 0, 5, 7, 3), 1.0, dA, 7, 0, dB, 5, 35, 0.0, dC2, 5, 0, config_id=10)
    torch.cuda.synchronize()
    assert np.array_equal(dC2.cpu().numpy(), c0)


def h_shape(kind, M, N, K, bt, ta=0, tb=0):
    import paper_2008_13145_amd as kt
    return kt.shape(M, N, K, bt, ta, tb)


def test_unaligned_and_padded_leading_dims(gpu):
    """Misaligned base pointers and odd leading dimensions take the scalar
    load path; results must still match."""
    h, torch = gpu
    M, N, K = 45, 51, 39
    a, b, c0 = _problem(M, N, K, 1, 0, 0, 99)
    ref = _oracle(a, b, c0, 1.0, 0.5)
    tol = _bound(a, b, c0, 1.0, 0.5)
    lda, ldb, ldc = K + 3, N + 1, N + 5
    bufA = torch.zeros(1 + M * lda, dtype=torch.float32, device="cuda")
    bufB = torch.zeros(1 + K * ldb, dtype=torch.float32, device="cuda")
    bufC = torch.zeros(1 + M * ldc, dtype=torch.float32, device="cuda")
    bufA[1:].view(M, lda)[:, :K] = torch.from_numpy(a[0]).cuda()
    bufB[1:].view(K, ldb)[:, :N] = torch.from_numpy(b[0]).cuda()
    cfgs = h.configs()
    for cfg in [cfgs.index(c) for c in [(8, 8, 1, 8), (32, 64, 2, 16), (64, 64, 4, 16), (128, 64, 8, 32)]]:
        bufC[1:].view(M, ldc)[:, :N] = torch.from_numpy(c0[0]).cuda()
        h.gemm_raw(0, h_shape(0, M, N, K, 1), 1.0, bufA.data_ptr() + 4, lda, 0,
                   bufB.data_ptr() + 4, ldb, 0, 0.5, bufC.data_ptr() + 4, ldc, 0, config_id=cfg)
        torch.cuda.synchronize()
        got = bufC[1:].view(M, ldc)[:, :N].cpu().numpy()
        assert np.all(np.abs(got - ref[0]) <= tol[0]), cfgs[cfg]


def test_invalid_arguments(gpu):
    import ctypes
    import paper_2008_13145_amd as kt
    h, torch = gpu
    d = torch.zeros(64, dtype=torch.float32, device="cuda")
    cases = [
        (kt.shape(-1, 4, 4), 4, 4, 4, -1),       # negative M
        (kt.shape(4, 4, 4), 3, 4, 4, -1),        # lda < K
        (kt.shape(4, 4, 4), 4, 3, 4, -1),        # ldb < N
        (kt.shape(4, 4, 4), 4, 4, 3, -1),        # ldc < N
        (kt.shape(4, 4, 4, 1, 2, 0), 4, 4, 4, -1),
    ]
    for shp, lda, ldb, ldc, want in cases:
        st = h.gemm_raw(0, shp, 1.0, d, lda, 16, d, ldb, 16, 0.0, d, ldc, 16, config_id=0, check=False)
        assert st == want
    st = h.gemm_raw(0, kt.shape(4, 4, 4), 1.0, d, 4, 0, d, 4, 0, 0.0, d, 4, 0,
                    config_id=h.num_kernels(), check=False)
    assert st == -1
    st = h.gemm_raw(0, kt.shape(4, 4, 4), 1.0, d, 4, 0, d, 4, 0, 0.0, d, 4, 0, config_id=-1, check=False)
    assert st == -4            # no selector fitted yet


def test_large_shape_sampled(gpu):
    """A large member of the sweep set, checked on 64 full rows and 64 full
    columns per batch item (the bound is per element)."""
    h, torch = gpu
    M, N, K, bt = 1536, 2000, 3000, 2
    ta, tb = 1, 0
    seed = 4242
    aop = synth.uniform_operand(synth.operand_seed(seed, 0), bt * M * K).reshape(bt, M, K)
    bop = synth.uniform_operand(synth.operand_seed(seed, 1), bt * K * N).reshape(bt, K, N)
    As = _stored(aop, ta)
    Bs = _stored(bop, tb)
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(M, 64, replace=False))
    cols = np.sort(rng.choice(N, 64, replace=False))
    ref_r, ref_c = og.gemm_sampled(M, N, K, bt, ta, tb, 1.0, 0.0, As, M, K * M, Bs, N, K * N,
                                   None, N, M * N, rows, cols)
    tol = 1e-5 * math.sqrt(K) * np.abs(aop).reshape(bt, -1).max(1) * np.abs(bop).reshape(bt, -1).max(1)
    dA, dB = torch.from_numpy(As).cuda(), torch.from_numpy(Bs).cuda()
    cfgs = h.configs()
    for c in [(128, 128, 8, 16), (128, 128, 8, 64), (64, 64, 4, 16), (16, 16, 2, 32)]:
        dC = torch.empty((bt, M, N), dtype=torch.float32, device="cuda")
        h.gemm(dA, dB, dC, ta, tb, 1.0, 0.0, config_id=cfgs.index(c))
        C = dC.cpu().numpy()
        for i in range(bt):
            assert np.all(np.abs(C[i][rows, :] - ref_r[i]) <= tol[i]), c
            assert np.all(np.abs(C[i][:, cols] - ref_c[i]) <= tol[i]), c


def test_batch_split_over_grids(gpu):
    """A batch whose flat (batch item, tile) grid exceeds the 32-bit work-item
    count of one launch (1024-thread work-groups, one tile per item) is split
    over several grids; every item must still be computed."""
    h, torch = gpu
    M, N, K = 2, 3, 5
    bt = 0xFFFFFFFF // 1024 + 7
    a = synth.uniform_operand(synth.operand_seed(77, 0), bt * M * K).reshape(bt, M, K)
    b = synth.uniform_operand(synth.operand_seed(77, 1), bt * K * N).reshape(bt, K, N)
    c0 = np.zeros((bt, M, N), np.float32)
    cfg = h.configs().index((128, 128, 4, 32))      # 16 waves = 1024 threads
    got = _run(h, torch, a, b, np.full_like(c0, np.nan), 0, 0, 1.0, 0.0, cfg)
    ref = _oracle(a, b, c0, 1.0, 0.0)
    assert not np.isnan(got).any()
    assert np.all(np.abs(got - ref) <= _bound(a, b, c0, 1.0, 0.0))
