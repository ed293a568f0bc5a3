"""Pins of the k-means pruning oracle (sections 4.1-4.2 of the paper)."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import kmeans as km


def _draws(seed, n_init, k):
    return km.restart_draws(synth.SplitMix64, seed, n_init, k)


def _partitions(n, k):
    """All labelings of n items into exactly k non-empty clusters (canonical)."""
    def rec(i, labels, used):
        if i == n:
            if used == k:
                yield list(labels)
            return
        for c in range(min(used + 1, k)):
            labels.append(c)
            yield from rec(i + 1, labels, max(used, c + 1))
            labels.pop()
    yield from rec(0, [], 0)


def _sse(X, labels, k):
    tot = Fraction(0)
    for c in range(k):
        m = X[labels == c]
        mean = [Fraction(int(v), len(m)) for v in m.sum(axis=0)]
        tot += sum((Fraction(int(x)) - mu) ** 2 for row in m for x, mu in zip(row, mean))
    return tot


def _is_fixed_point(X, res):
    C = res["centroids"]
    lab, dist = km.assign(X, C)
    if not np.array_equal(lab, res["labels"]):
        return False
    for j in range(C.shape[0]):
        m = X[lab == j]
        if len(m):
            want = [(2 * int(s) + len(m)) // (2 * len(m)) for s in m.sum(axis=0)]
            if list(C[j]) != want:
                return False
    return int(dist.sum()) == res["inertia"]


def test_brute_force_planted_tiny():
    rng = np.random.default_rng(3)
    for trial in range(20):
        k = 2 + trial % 2
        n = 6 + trial % 3
        d = 2 + trial % 3
        centres = rng.integers(0, 3, size=(k, d)) * 20000
        lab = np.array([i % k for i in range(n)])
        X = centres[lab] + rng.integers(-300, 300, size=(n, d)) + 1000
        res = km.kmeans(X, k, _draws(100 + trial, 10, k))
        assert _is_fixed_point(X, res)
        if len({tuple(c) for c in centres}) == k:
            best = min(_partitions(n, k), key=lambda p: _sse(X, np.array(p), k))
            # same partition up to relabeling
            got = res["labels"]
            pairs = {(int(a), int(b)) for a, b in zip(best, got)}
            assert len(set(best)) == k and len(set(int(v) for v in got)) == k
            assert len(pairs) == k


def test_every_result_is_a_fixed_point_random():
    rng = np.random.default_rng(4)
    for trial in range(30):
        n, d, k = int(rng.integers(3, 9)), int(rng.integers(1, 5)), int(rng.integers(1, 4))
        k = min(k, n)
        X = rng.integers(0, 65536, size=(n, d))
        res = km.kmeans(X, k, _draws(trial, 5, k))
        assert _is_fixed_point(X, res)


def test_planted_q16_clusters_recover_configs():
    rng = np.random.default_rng(5)
    d, k, per = 40, 4, 30
    groups = [3, 17, 25, 38]
    rows, truth = [], []
    for gi, g in enumerate(groups):
        for _ in range(per):
            r = 13000 + rng.integers(-500, 500, size=d)
            r[g] = 65535
            rows.append(r)
            truth.append(gi)
    X = np.array(rows)
    res = km.kmeans(X, k, _draws(7, 10, k))
    lab = res["labels"]
    assert len({(t, int(l)) for t, l in zip(truth, lab)}) == k
    assert sorted(km.centroids_to_configs(res["centroids"])) == groups


def test_k_one_is_rounded_mean():
    rng = np.random.default_rng(6)
    X = rng.integers(0, 65536, size=(23, 9))
    res = km.kmeans(X, 1, _draws(1, 3, 1))
    n = X.shape[0]
    for f in range(X.shape[1]):
        exact = Fraction(int(X[:, f].sum()), n)
        c = int(res["centroids"][0, f])
        assert c - Fraction(1, 2) <= exact < c + Fraction(1, 2)


def test_k_equals_n_distinct_gives_zero_inertia():
    rng = np.random.default_rng(8)
    X = rng.permutation(np.arange(0, 65536, 997))[:12].reshape(6, 2)
    res = km.kmeans(X, 6, _draws(2, 4, 6))
    assert res["inertia"] == 0


def test_kmeanspp_first_centre_and_zero_mass():
    X = np.array([[5, 5]] * 4 + [[9, 9]])
    draws = [12, 0, 0]
    idx = km.kmeanspp_init(X, 3, draws)
    assert idx[0] == 12 % 5
    # after picking rows 2 (=[5,5]) and 4 (=[9,9]) all mass is zero -> lowest unused row
    assert list(idx) == [2, 4, 0]


def test_kmeanspp_draw_selects_by_cumulative_mass():
    X = np.array([[0], [1], [3]])          # D^2 to row 0: 0, 1, 9 (cumulative 0, 1, 10)
    assert list(km.kmeanspp_init(X, 2, [0, 0])) == [0, 1]     # r = 0 -> first cum > 0
    assert list(km.kmeanspp_init(X, 2, [0, 1])) == [0, 2]     # r = 1 -> first cum > 1
    assert list(km.kmeanspp_init(X, 2, [0, 9])) == [0, 2]


def test_sklearn_cross_check_separated():
    sk = pytest.importorskip("sklearn.cluster")
    rng = np.random.default_rng(9)
    centres = np.array([[0, 0, 0], [40000, 0, 0], [0, 40000, 40000]])
    X = np.concatenate([c + rng.integers(0, 2000, size=(25, 3)) for c in centres])
    res = km.kmeans(X, 3, _draws(11, 1, 3))
    init = X[res["init"]].astype(np.float64)
    ref = sk.KMeans(n_clusters=3, init=init, n_init=1).fit(X.astype(np.float64))
    assert np.array_equal(ref.labels_, res["labels"])


def test_centroid_to_config_dedupe_and_topn():
    C = np.array([[10, 50, 50, 0], [0, 60, 10, 5], [1, 70, 2, 3]])
    # centroid 0 -> config 1 (first of the tied maxima), centroid 1 -> 1 taken -> 2,
    # centroid 2 -> 1 taken, 0 next (value 3 at config 3 beats 2 at config 2? no: 3 > 2 > 1)
    assert km.centroids_to_configs(C) == [1, 2, 3]
    Xq = np.array([[65535, 1, 2], [3, 65535, 1], [65535, 0, 0], [0, 0, 65535]])
    assert km.top_n(Xq, 2) == [0, 1]
    assert km.top_n(Xq, 3) == [0, 1, 2]
