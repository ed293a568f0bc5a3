"""Pins of the FP64 GEMM oracle (section 3 of the paper) against exact
arithmetic, closed forms and invariants."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import gemm as og


def _store(opmat, trans):
    """Row-major storage of an op() matrix for the given transpose flag."""
    return np.ascontiguousarray(opmat.T if trans else opmat)


def _call(a_op, b_op, ta, tb, alpha, beta, c0):
    """a_op: (batch, M, K), b_op: (batch, K, N) in op() orientation."""
    bt, M, K = a_op.shape
    N = b_op.shape[2]
    As = np.stack([_store(a_op[i], ta) for i in range(bt)])
    Bs = np.stack([_store(b_op[i], tb) for i in range(bt)])
    lda = As.shape[2]
    ldb = Bs.shape[2]
    return og.gemm(M, N, K, bt, ta, tb, alpha, beta, As, lda, As.shape[1] * lda,
                   Bs, ldb, Bs.shape[1] * ldb, c0, N, M * N)


def _exact(a_op, b_op, alpha, beta, c0):
    bt, M, K = a_op.shape
    N = b_op.shape[2]
    out = np.empty((bt, M, N), dtype=object)
    for b in range(bt):
        for i in range(M):
            for j in range(N):
                s = sum((Fraction(float(a_op[b, i, k])) * Fraction(float(b_op[b, k, j]))
                         for k in range(K)), Fraction(0))
                v = Fraction(alpha) * s
                if beta != 0:
                    v += Fraction(beta) * Fraction(float(c0[b, i, j]))
                out[b, i, j] = v
    return out


@pytest.mark.parametrize("ta,tb", synth.LAYOUTS)
def test_brute_force_tiny_exact(ta, tb):
    # FP32 values on a 2**-23 grid: every partial sum of <= 5 products and the
    # alpha/beta combination are exact in FP64, so the oracle must equal the
    # rational result exactly.
    seed = 11
    for (M, N, K) in itertools.product((1, 2, 3, 5), (1, 2, 4), (1, 3, 5)):
        for bt in (1, 2):
            a = synth.uniform_operand(synth.operand_seed(seed, 0), bt * M * K).reshape(bt, M, K)
            b = synth.uniform_operand(synth.operand_seed(seed, 1), bt * K * N).reshape(bt, K, N)
            c0 = synth.uniform_operand(synth.operand_seed(seed, 2), bt * M * N).reshape(bt, M, N)
            seed += 1
            for alpha, beta in ((1.0, 0.0), (-0.5, 2.0), (2.0, 1.0), (0.0, -0.5)):
                got = _call(a, b, ta, tb, alpha, beta, c0)
                ex = _exact(a, b, alpha, beta, c0)
                for idx in np.ndindex(got.shape):
                    assert Fraction(float(got[idx])) == ex[idx], (M, N, K, bt, alpha, beta, idx)


@pytest.mark.parametrize("ta,tb", synth.LAYOUTS)
def test_identity(ta, tb):
    M = K = 37
    N = 23
    a = np.eye(M, dtype=np.float32)[None]
    b = synth.uniform_operand(5, K * N).reshape(1, K, N)
    got = _call(a, b, ta, tb, 1.0, 0.0, None)
    assert np.array_equal(got[0], b[0].astype(np.float64))


@pytest.mark.parametrize("ta,tb", synth.LAYOUTS)
def test_closed_forms(ta, tb):
    M, N, K = 19, 13, 41
    i = np.arange(M)[:, None]
    j = np.arange(N)[None, :]
    # rank one: A_ik = u_i, B_kj = v_j  =>  C_ij = K u_i v_j
    u = (np.arange(M) % 7 - 3).astype(np.float32)
    v = (np.arange(N) % 5 - 2).astype(np.float32)
    a = np.repeat(u[:, None], K, axis=1)[None]
    b = np.repeat(v[None, :], K, axis=0)[None]
    got = _call(a, b, ta, tb, 1.0, 0.0, None)[0]
    assert np.array_equal(got, K * u[:, None].astype(np.float64) * v[None, :])
    # A_ik = i + k, B_kj = j + k  =>  C_ij = K i j + (i + j) K(K-1)/2 + (K-1)K(2K-1)/6
    kk = np.arange(K)
    a = (np.arange(M)[:, None] + kk[None, :]).astype(np.float32)[None]
    b = (kk[:, None] + np.arange(N)[None, :]).astype(np.float32)[None]
    got = _call(a, b, ta, tb, 1.0, 0.0, None)[0]
    want = K * i * j + (i + j) * K * (K - 1) // 2 + (K - 1) * K * (2 * K - 1) // 6
    assert np.array_equal(got, want.astype(np.float64))


def test_beta_zero_ignores_nan_and_k_zero():
    M, N, K = 5, 6, 7
    a = synth.uniform_operand(1, M * K).reshape(1, M, K)
    b = synth.uniform_operand(2, K * N).reshape(1, K, N)
    c0 = np.full((1, M, N), np.nan, dtype=np.float32)
    got = _call(a, b, 0, 0, 1.5, 0.0, c0)
    assert not np.isnan(got).any()
    c0 = synth.uniform_operand(3, M * N).reshape(1, M, N)
    got = og.gemm(M, N, 0, 1, 0, 0, 2.0, -0.5, a, 1, 0, b, N, 0, c0, N, M * N)
    assert np.array_equal(got[0], -0.5 * c0[0].astype(np.float64))


def test_transpose_equivalence_and_batch_strides():
    M, N, K, bt = 9, 11, 17, 3
    a = synth.uniform_operand(7, bt * M * K).reshape(bt, M, K)
    b = synth.uniform_operand(8, bt * K * N).reshape(bt, K, N)
    ref = _call(a, b, 0, 0, 1.0, 0.0, None)
    for ta, tb in synth.LAYOUTS:
        assert np.array_equal(_call(a, b, ta, tb, 1.0, 0.0, None), ref)
    for i in range(bt):
        one = _call(a[i:i + 1], b[i:i + 1], 0, 0, 1.0, 0.0, None)
        assert np.array_equal(one[0], ref[i])
    # padded leading dimensions and batch strides
    lda, ldb = K + 3, N + 5
    As = np.zeros((bt, M + 1, lda), dtype=np.float32)
    As[:, :M, :K] = a
    Bs = np.zeros((bt, K, ldb), dtype=np.float32)
    Bs[:, :, :N] = b
    got = og.gemm(M, N, K, bt, 0, 0, 1.0, 0.0, As, lda, (M + 1) * lda, Bs, ldb, K * ldb)
    assert np.array_equal(got, ref)


def test_sampled_matches_full():
    M, N, K, bt = 33, 29, 50, 2
    a = synth.uniform_operand(9, bt * M * K)
    b = synth.uniform_operand(10, bt * K * N)
    c0 = synth.uniform_operand(11, bt * M * N)
    full = og.gemm(M, N, K, bt, 1, 0, 0.75, -2.0, a, M, M * K, b, N, K * N, c0, N, M * N)
    rows = np.array([0, 5, 32])
    cols = np.array([3, 28])
    r, c = og.gemm_sampled(M, N, K, bt, 1, 0, 0.75, -2.0, a, M, M * K, b, N, K * N,
                           c0, N, M * N, rows, cols)
    assert np.array_equal(r, full[:, rows, :])
    assert np.array_equal(c, full[:, :, cols])
