"""Pins of the cluster -> kernel rules of section 4.2 (oracle.represent):
hand-worked clusters where the arithmetic and the geometric mean disagree,
the fixed-point logarithm against a 50-digit decimal evaluation, and the
geometric-mean rule against exact products of fractions."""
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np

from oracle import represent as orep


def test_worked_clusters():
    Xq = np.array([
        [65535, 30000, 100, 0],     # cluster 0
        [1, 30000, 100, 0],         # cluster 0
        [100, 50000, 65535, 10],    # cluster 1
        [100, 50000, 60000, 10],    # cluster 1
        [0, 0, 0, 65535],           # cluster 2
    ])
    labels = [0, 0, 1, 1, 2]
    # means: c0 (32768, 30000, 100, 0) -> 0; c1 (100, 50000, 62768, 10) -> 2;
    # c2 -> 3
    assert orep.mean_representatives(Xq, labels, 3, 3) == [0, 2, 3]
    # geometric means: c0 config 0 = sqrt(65535 * 1) ~ 256 < 30000 -> 1;
    # c1 config 2 = sqrt(65535 * 60000) ~ 62707 -> 2; c2 -> 3
    assert orep.geomean_representatives(Xq, labels, 3, 3) == [1, 2, 3]


def test_distinct_picks_and_fill():
    Xq = np.array([[65535, 60000, 0], [65535, 50000, 0], [1000, 2000, 3000]])
    # both of the first two clusters prefer configuration 0: the second takes
    # its next best
    assert orep.mean_representatives(Xq, [0, 1, 2], 3, 3) == [0, 1, 2]
    # one non-empty cluster of two (cluster 1 empty): fill by the column sums
    # of the whole table (132070, 112000, 3000)
    assert orep.mean_representatives(Xq, [0, 0, 0], 2, 2) == [0, 1]
    # geometric: column log-sums rank configuration 1 (60000*50000*2000)
    # above 0 (65535*65535*1000) above 2 (1*1*3000)
    assert orep.geomean_representatives(Xq, [2, 2, 2], 3, 3) == [1, 0, 2]


def test_log_table_against_decimal():
    L = orep.log2_table()
    assert L[65535] == 0 and L[0] == L[1]
    assert np.all(np.diff(L[1:]) > 0)
    getcontext().prec = 50
    ln2 = Decimal(2).ln()
    checked = 0
    for q in list(range(1, 65536, 97)) + [1, 2, 3, 32767, 32768, 65534]:
        exact = Decimal(2 ** 32) * (Decimal(q) / Decimal(65535)).ln() / ln2
        frac = exact - exact.to_integral_value(rounding="ROUND_FLOOR")
        if abs(frac - Decimal("0.5")) < Decimal("1e-5"):
            continue            # too close to a rounding tie to pin
        assert L[q] == int(exact.to_integral_value(rounding="ROUND_HALF_EVEN")), q
        checked += 1
    assert checked > 600


def test_geomean_rule_equals_exact_products():
    rng = np.random.default_rng(3)
    for trial in range(30):
        n, d = int(rng.integers(1, 6)), int(rng.integers(2, 7))
        Xq = rng.integers(0, 65536, (n, d))
        Xq[rng.random((n, d)) < 0.2] = 0
        prods = [np.prod([Fraction(max(int(v), 1), 65535) for v in Xq[:, j]]) for j in range(d)]
        best = max(range(d), key=lambda j: (prods[j], -j))
        srt = sorted(prods, reverse=True)
        if len(srt) > 1 and srt[0] != srt[1] and float(srt[1] / srt[0]) > 1 - 1e-8:
            continue            # products too close for the fixed-point logarithm
        assert orep.geomean_representatives(Xq, [0] * n, 1, 1) == [best], trial


def test_tree_pruning_is_the_mean_rule_on_its_leaves():
    # decision-tree pruning (section 4.1) picks by the rounded leaf means,
    # filled by column sums: the mean rule applied to its leaf labels
    from oracle import prune_tree as opt
    rng = np.random.default_rng(5)
    for trial in range(5):
        n, d, k = 40, 12, int(rng.integers(2, 7))
        F = np.stack([rng.integers(16, 4096, n), rng.integers(16, 4096, n), rng.integers(16, 4096, n),
                      rng.integers(1, 64, n), rng.integers(0, 2, n), rng.integers(0, 2, n)], axis=1)
        X = rng.integers(0, 65536, (n, d))
        labels, n_leaves = opt.leaf_labels(F, X, k)
        assert orep.mean_representatives(X, labels, n_leaves, k) == opt.prune(F, X, k)
