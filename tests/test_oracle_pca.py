"""Pins of the PCA oracle (paper section 4.1, "PCA and k-means clustering")
against facts it does not compute itself: planted axes and variances of a
rotated diagonal covariance, orthonormality, the total variance summed from
the data, exact reconstruction at full rank, a hand-worked two-dimensional
case and a hand-worked quantization."""
import math

import numpy as np
import pytest

from oracle import kmeans as okm
from oracle import normalize as onorm
from oracle import pca as opca

import synth


def _planted(n, d, sig, seed):
    """Points whose centred sample covariance is exactly R diag(sig^2/(n-1)) R^T:
    Q has orthonormal columns orthogonal to the all-ones vector."""
    rng = np.random.default_rng(seed)
    R, _ = np.linalg.qr(rng.standard_normal((d, d)))
    Q, _ = np.linalg.qr(np.concatenate([np.ones((n, 1)), rng.standard_normal((n, d))], axis=1))
    Q = Q[:, 1:d + 1]
    mu = rng.uniform(-1, 1, d)
    return mu + (Q * sig) @ R.T, R, mu


@pytest.mark.parametrize("n,d,seed", [(40, 5, 1), (200, 12, 2), (14, 13, 3)])
def test_planted_axes_and_variances(n, d, seed):
    sig = np.linspace(3.0, 0.5, d) ** 2 + np.arange(d)[::-1] * 0.01
    X, R, mu = _planted(n, d, sig, seed)
    P = opca.pca(X, d)
    assert np.allclose(P["mean"], mu, atol=1e-12)
    assert np.allclose(P["variances"], sig ** 2 / (n - 1), rtol=1e-10)
    for i in range(d):
        # each component is a planted axis up to sign
        c = float(np.dot(P["components"][i], R[:, i]))
        assert abs(abs(c) - 1.0) < 1e-9


def test_components_orthonormal_and_signed():
    rng = np.random.default_rng(7)
    X = rng.uniform(0, 1, (60, 9)) @ rng.uniform(-1, 1, (9, 9))
    P = opca.pca(X, 9)
    V = P["components"]
    assert np.allclose(V @ V.T, np.eye(9), atol=1e-12)
    for v in V:
        a = np.abs(v)
        first = int(np.argmax(a >= (1 - 1e-9) * a.max()))
        assert v[first] > 0


def test_total_variance_from_the_data():
    rng = np.random.default_rng(8)
    X = rng.uniform(0, 1, (50, 6))
    P = opca.pca(X, 2)
    # trace of the covariance summed column by column, without the eigen-solver
    tot = sum(float(np.sum((X[:, j] - X[:, j].mean()) ** 2)) for j in range(6)) / 49
    assert math.isclose(float(P["variances"].sum()), tot, rel_tol=1e-12)
    assert math.isclose(P["explained"], float(P["variances"][:2].sum()) / tot, rel_tol=1e-12)
    assert all(P["variances"][i] >= P["variances"][i + 1] for i in range(5))


def test_full_rank_reconstruction_is_exact():
    rng = np.random.default_rng(9)
    X = rng.uniform(0, 1, (30, 7))
    P = opca.pca(X, 7)
    assert np.allclose(P["mean"] + P["Z"] @ P["components"], X, atol=1e-12)


def test_points_on_a_line():
    # (t, 2t): one component along (1, 2)/sqrt(5) with all the variance
    t = np.arange(-3.0, 4.0)
    X = np.stack([t, 2 * t], axis=1)
    P = opca.pca(X, 1)
    assert np.allclose(P["components"][0], np.array([1.0, 2.0]) / math.sqrt(5), atol=1e-12)
    assert math.isclose(P["variances"][0], 5 * np.var(t, ddof=1), rel_tol=1e-12)
    assert abs(P["variances"][1]) < 1e-12
    assert math.isclose(P["explained"], 1.0, rel_tol=1e-12)
    assert np.allclose(P["Z"][:, 0], t * math.sqrt(5), atol=1e-12)


def test_quantization_worked_example():
    Z = np.array([[-1.0, 0.0], [1.0, 0.5]])
    U, lo, span = opca.quantize(Z)
    assert (lo, span) == (-1.0, 2.0)
    # 0.5 * 65535 = 32767.5 rounds to even 32768; 0.75 * 65535 = 49151.25
    assert U.tolist() == [[0, 32768], [65535, 49151]]
    U0, _, s0 = opca.quantize(np.full((3, 2), 0.25))
    assert s0 == 0.0 and not U0.any()


def test_centroid_read_back_at_full_rank():
    # a centroid equal to a quantized point reads back to that point within
    # the quantization step
    rng = np.random.default_rng(10)
    X = rng.integers(0, 65536, (25, 6)).astype(np.float64) / 65535
    P = opca.pca(X, 6)
    U, lo, span = opca.quantize(P["Z"])
    for i in range(25):
        q = opca.centroid_q16(U[i], lo, span, P["mean"], P["components"])
        # half a quantization step per coordinate, in Q16 units, plus rounding
        step = span * math.sqrt(6) / 2 + 1
        assert np.all(np.abs(q - np.rint(65535 * X[i])) <= step)


def test_prune_pca_planted_clusters():
    # rows of group g are fastest at configuration g: every rule must find
    # one configuration per group
    rng = np.random.default_rng(11)
    groups, d, per = 4, 10, 12
    T = rng.integers(3000, 4000, (groups * per, d)).astype(np.int64)
    for g in range(groups):
        T[g * per:(g + 1) * per, g] = 1000
    draws = okm.restart_draws(synth.SplitMix64, 5, 4, groups)
    for rep in (opca.REP_CENTROID, opca.REP_GEOMEAN):
        for m in (2, 3, 10):
            r = opca.prune_pca(T, groups, onorm.RELATIVE, m, rep, draws)
            assert sorted(r["chosen"]) == list(range(groups)), (rep, m, r["chosen"])
