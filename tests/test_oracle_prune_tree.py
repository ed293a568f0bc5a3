"""Pins of the decision-tree pruning oracle: brute force over every single
split on tiny inputs (the first split is the exhaustive optimum of the
summed squared error), the one-leaf case (column means), a planted two-regime
table, constant features (no split possible, fill rule) and a partition
invariant."""
import itertools
import math

import numpy as np

from oracle import prune_tree as pt


def _sse(X, rows):
    if not rows:
        return 0.0
    Y = X[rows].astype(np.float64)
    return float(((Y - Y.mean(axis=0)) ** 2).sum())


def test_first_split_is_the_brute_force_optimum():
    """For k = 2 the tree's only split minimises the children's summed squared
    error over every (feature, threshold) partition, found by enumeration."""
    rng = np.random.default_rng(5)
    for trial in range(6):
        n, d = 9, 4
        F = np.column_stack([rng.integers(1, 50, n), rng.integers(1, 6, n), rng.integers(0, 2, n)])
        X = rng.integers(0, 65536, size=(n, d))
        nodes, pre = pt.fit(F, X, 2)
        root = nodes[0]
        best = None
        for f in range(F.shape[1]):
            vals = sorted(set(F[:, f].tolist()))
            for a, b in zip(vals, vals[1:]):
                left = [i for i in range(n) if F[i, f] <= a]
                right = [i for i in range(n) if F[i, f] > a]
                e = _sse(X, left) + _sse(X, right)
                if best is None or e < best[0] - 1e-6:
                    best = (e, f, math.isqrt(a * b))
        assert (root["feature"], root["threshold"]) == best[1:]
        left = nodes[root["left"]]["rows"]
        assert abs(_sse(X, left) + _sse(X, nodes[root["right"]]["rows"]) - best[0]) < 1e-6


def test_one_leaf_is_the_column_mean_argmax():
    rng = np.random.default_rng(6)
    X = rng.integers(0, 65536, size=(30, 12))
    F = rng.integers(1, 100, size=(30, 6))
    assert pt.prune(F, X, 1) == [int(np.argmax(X.sum(axis=0)))]


def test_planted_regimes():
    """Rows with K <= 100 are best on configuration 3, the others on 7; two
    leaves recover exactly those two."""
    rng = np.random.default_rng(7)
    n, d = 40, 10
    F = np.column_stack([rng.integers(16, 4096, n), rng.integers(16, 4096, n),
                         np.where(np.arange(n) % 2 == 0, rng.integers(16, 100, n), rng.integers(200, 4000, n)),
                         rng.integers(1, 64, n), rng.integers(0, 2, n), rng.integers(0, 2, n)])
    X = rng.integers(0, 20000, size=(n, d))
    X[F[:, 2] <= 100, 3] = 65535
    X[F[:, 2] > 100, 7] = 65535
    nodes, pre = pt.fit(F, X, 2)
    assert nodes[0]["feature"] == 2
    assert sorted(nodes[nodes[0]["left"]]["rows"]) == [i for i in range(n) if F[i, 2] <= 100]
    assert pt.prune(F, X, 2) == [3, 7]


def test_constant_features_fill_from_column_sums():
    X = np.array([[10, 50, 30, 40], [20, 60, 10, 45]], dtype=np.int64)
    F = np.ones((2, 6), dtype=np.int64)
    # one leaf (no feature varies): its mean picks 1, then column sums 3 (85), 2 (40), 0 (30)
    assert pt.prune(F, X, 3) == [1, 3, 2]


def test_leaves_partition_rows_and_follow_thresholds():
    rng = np.random.default_rng(8)
    F = rng.integers(1, 300, size=(80, 6))
    X = rng.integers(0, 65536, size=(80, 20))
    nodes, pre = pt.fit(F, X, 6)
    assert len(pre) == 6
    rows = sorted(itertools.chain.from_iterable(nodes[i]["rows"] for i in pre))
    assert rows == list(range(80))
    for nd in nodes:
        if nd["feature"] >= 0:
            assert all(F[i, nd["feature"]] <= nd["threshold"] for i in nodes[nd["left"]]["rows"])
            assert all(F[i, nd["feature"]] > nd["threshold"] for i in nodes[nd["right"]]["rows"])
    ch = pt.prune(F, X, 6)
    assert len(set(ch)) == 6
