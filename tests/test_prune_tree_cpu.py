"""Decision-tree pruning in the library (host code, no GPU) against the
oracle, pick for pick: seeded random tables, planted regimes, constant
features, and the FP32 sweep table's training rows under every
normalization (normalized by the oracle)."""
import numpy as np
import pytest

import synth
from oracle import normalize as onorm
from oracle import prune_tree as opt


def _shapes(F):
    return [tuple(int(v) for v in row) for row in F]


@pytest.mark.parametrize("n,d,k,seed", [(60, 12, 4, 1), (200, 40, 8, 2), (333, 97, 15, 3), (5, 9, 5, 4)])
def test_random_tables(kt, n, d, k, seed):
    rng = np.random.default_rng(seed)
    F = np.column_stack([rng.integers(16, 4097, n), rng.integers(16, 4097, n), rng.integers(16, 4097, n),
                         rng.integers(1, 65, n), rng.integers(0, 2, n), rng.integers(0, 2, n)])
    X = rng.integers(0, 65536, size=(n, d))
    h = kt.Handle(-1)
    assert h.prune_tree(_shapes(F), X, k) == opt.prune(F, X, k)


def test_constant_features_and_duplicates(kt):
    h = kt.Handle(-1)
    X = np.array([[10, 50, 30, 40], [20, 60, 10, 45]], dtype=np.int64)
    F = np.ones((2, 6), dtype=np.int64)
    assert h.prune_tree(_shapes(F), X, 3) == opt.prune(F, X, 3) == [1, 3, 2]
    rng = np.random.default_rng(9)
    F = np.repeat(rng.integers(1, 50, size=(4, 6)), 5, axis=0)
    X = rng.integers(0, 65536, size=(20, 8))
    assert h.prune_tree(_shapes(F), X, 6) == opt.prune(F, X, 6)


@pytest.mark.parametrize("norm", [0, 1, 2, 3])
def test_sweep_table_training_rows(kt, norm):
    from paper_2008_13145_amd import tune
    T, P, C, meta = tune.load_table(tune.DEFAULT_TABLE)
    train, _ = synth.train_test_split()
    rows = synth.rows_of_shapes(train)
    Xq = onorm.normalize(T[rows].astype(np.int64), norm)
    F = P[rows]
    h = kt.Handle(-1)
    for k in (4, 8):
        assert h.prune_tree(_shapes(F), Xq, k) == opt.prune(F, Xq, k)


def test_rejects_bad_arguments(kt):
    h = kt.Handle(-1)
    X = np.zeros((3, 4), dtype=np.uint16)
    with pytest.raises(kt.KtError):
        h.prune_tree([(1, 1, 1, 1, 0, 0)] * 3, X, 5)
    with pytest.raises(kt.KtError):
        h.prune_tree([(1, 1, 1, 1, 0, 0)] * 3, np.zeros((3, 300), dtype=np.uint16), 2)
