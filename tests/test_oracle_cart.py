"""Pins of the decision-tree oracle (section 5.1 of the paper)."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import cart


def _rand_data(rng, n, n_classes, card=40):
    X = np.stack([rng.integers(16, 4097, size=n), rng.integers(16, 4097, size=n),
                  rng.integers(16, 4097, size=n), rng.integers(1, 65, size=n),
                  rng.integers(0, 2, size=n), rng.integers(0, 2, size=n)], axis=1)
    y = rng.integers(0, n_classes, size=n)
    return X, y


def _leaves(tree):
    return [i for i, f in enumerate(tree["feature"]) if f < 0]


def _route(tree, X):
    out = []
    for x in X:
        node = 0
        while tree["feature"][node] >= 0:
            node = tree["left"][node] if x[tree["feature"][node]] <= tree["threshold"][node] \
                else tree["right"][node]
        out.append(node)
    return np.array(out)


def _node_depths(tree):
    d = {0: 0}
    for i in range(len(tree["feature"])):
        if tree["feature"][i] >= 0:
            d[tree["left"][i]] = d[i] + 1
            d[tree["right"][i]] = d[i] + 1
    return d


def test_separable_toy_depth_one():
    X = np.array([[m, 64, 64, 1, 0, 0] for m in (16, 100, 300, 499, 501, 900, 4096)])
    y = (X[:, 0] > 500).astype(int)
    t = cart.fit(X, y, 2, None, 1)
    assert t["feature"][0] == 0 and t["threshold"][0] == math.isqrt(499 * 501)
    assert cart.depth(t) == 1
    assert np.array_equal(cart.predict(t, X), y)


@pytest.mark.parametrize("variant", ["A", "B", "C"])
def test_invariants(variant):
    max_depth, min_leaf = cart.TREE_PARAMS[variant]
    rng = np.random.default_rng(12)
    X, y = _rand_data(rng, 300, 5)
    t = cart.fit(X, y, 5, max_depth, min_leaf)
    leaf_of = _route(t, X)
    counts = np.bincount(leaf_of, minlength=len(t["feature"]))
    assert sum(counts[l] for l in _leaves(t)) == len(y)
    assert all(counts[l] >= min_leaf for l in _leaves(t))
    depths = _node_depths(t)
    if max_depth is not None:
        assert max(depths.values()) <= max_depth
    for l in _leaves(t):
        c = np.bincount(y[leaf_of == l], minlength=5)
        assert t["cls"][l] == int(np.argmax(c))       # majority, lowest class on ties
    # thresholds sit in [a, b) of two present values at that node: x <= t goes left
    for i, f in enumerate(t["feature"]):
        if f >= 0:
            assert t["left"][i] == i + 1                 # pre-order, left first


def test_tree_a_fits_tie_free_data():
    rng = np.random.default_rng(13)
    X, y = _rand_data(rng, 250, 4)
    _, first = np.unique(X, axis=0, return_index=True)
    X, y = X[np.sort(first)], y[np.sort(first)]
    t = cart.fit(X, y, 4, None, 1)
    assert np.array_equal(cart.predict(t, X), y)


def _gini_weighted(y, mask, n_classes):
    """Weighted Gini impurity n_L*G_L + n_R*G_R as a Fraction."""
    tot = Fraction(0)
    for part in (y[mask], y[~mask]):
        n = len(part)
        c = np.bincount(part, minlength=n_classes)
        tot += n - Fraction(int((c * c).sum()), n)
    return tot


def test_root_split_brute_force():
    rng = np.random.default_rng(14)
    for trial in range(40):
        n = int(rng.integers(4, 11))
        X = rng.integers(1, 9, size=(n, 6))
        y = rng.integers(0, 3, size=n)
        min_leaf = 1 + trial % 2
        t = cart.fit(X, y, 3, None, min_leaf)
        # enumerate every (feature, threshold between distinct values), first minimum wins
        best = None
        for f in range(6):
            vals = sorted(set(X[:, f].tolist()))
            for a, b in zip(vals, vals[1:]):
                thr = math.isqrt(a * b)
                mask = X[:, f] <= thr
                if mask.sum() < min_leaf or (~mask).sum() < min_leaf:
                    continue
                g = _gini_weighted(y, mask, 3)
                if best is None or g < best[0]:
                    best = (g, f, thr)
        c = np.bincount(y, minlength=3)
        parent = n - Fraction(int((c * c).sum()), n)
        if best is None or not best[0] < parent or (c > 0).sum() < 2:
            assert t["feature"][0] == -1
        else:
            assert (t["feature"][0], t["threshold"][0]) == (best[1], best[2]), trial


def test_sklearn_cross_check_root_impurity():
    sk = pytest.importorskip("sklearn.tree")
    rng = np.random.default_rng(15)
    X, y = _rand_data(rng, 400, 4)
    t = cart.fit(X, y, 4, 1, 1)
    ref = sk.DecisionTreeClassifier(criterion="gini", max_depth=1, min_samples_leaf=1).fit(X, y)
    tr = ref.tree_
    n = len(y)
    sk_child = (tr.impurity[1] * tr.n_node_samples[1] + tr.impurity[2] * tr.n_node_samples[2])
    mask = X[:, t["feature"][0]] <= t["threshold"][0]
    ours = float(_gini_weighted(y, mask, 4))
    assert abs(ours - sk_child) < 1e-9 * n


def test_labels_from_times_ties_and_invalid():
    T = np.array([[5, 3, 3, 9], [7, -1, 8, 2], [4, 4, 4, 4]])
    assert cart.labels_from_times(T, [0, 1, 2]).tolist() == [1, 0, 0]
    assert cart.labels_from_times(T, [3, 2]).tolist() == [1, 0, 0]
