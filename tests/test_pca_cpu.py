"""Host-side library calls against the oracle, on the CPU (a handle without
a device): principal components and their quantization (kt_pca), the
cluster -> kernel rules of section 4.2 (kt_representatives), decision-tree
leaves (kt_prune_tree_leaves) and the evaluation of section 4.3
(kt_evaluate), the last on the committed MI355X timing table."""
import numpy as np
import pytest

import synth
from oracle import normalize as onorm
from oracle import pca as opca
from oracle import prune_tree as opt
from oracle import regret as oreg
from oracle import represent as orep


@pytest.fixture(scope="module")
def host(kt):
    h = kt.Handle(-1)
    yield h
    h.close()


@pytest.fixture(scope="module")
def table():
    from paper_2008_13145_amd import tune
    T, P, C, meta = tune.load_table(tune.DEFAULT_TABLE)
    train, test = synth.train_test_split()
    return T, [tuple(int(v) for v in p) for p in P], synth.rows_of_shapes(train), \
        synth.rows_of_shapes(test)


def _pca_agree(got, ref, m):
    d = ref["components"].shape[1]
    assert np.allclose(got["mean"], ref["mean"], rtol=0, atol=1e-13)
    assert np.allclose(got["variances"], ref["variances"], rtol=1e-9, atol=1e-14)
    assert np.allclose(got["components"], ref["components"], rtol=0, atol=1e-9)
    assert abs(got["explained"] - ref["explained"]) < 1e-12
    assert got["components"].shape == (m, d)


def test_log_table_bitwise(host):
    assert np.array_equal(host.log2_q16_table(), orep.log2_table())


@pytest.mark.parametrize("norm", [onorm.RELATIVE, onorm.STDCUT, onorm.SIGMOID])
def test_pca_on_the_measured_table(host, table, norm):
    T, _, tr, _ = table
    Xq = onorm.normalize(T[tr], norm)
    for m in (8, 16):
        got = host.pca(Xq, m)
        ref = opca.pca(Xq.astype(np.float64) / 65535.0, m)
        _pca_agree(got, ref, m)
        U, lo, span = opca.quantize(ref["Z"])
        assert abs(got["lo"] - lo) < 1e-12 and abs(got["span"] - span) < 1e-12
        diff = np.abs(got["U"].astype(np.int64) - U.astype(np.int64))
        assert not diff.any(), int((diff > 0).sum())


def test_pca_random_tables(host):
    rng = np.random.default_rng(21)
    for trial in range(6):
        n, d = int(rng.integers(5, 80)), int(rng.integers(2, 40))
        m = int(rng.integers(1, d + 1))
        Xq = rng.integers(0, 65536, (n, d)).astype(np.uint16)
        got = host.pca(Xq, m)
        ref = opca.pca(Xq.astype(np.float64) / 65535.0, m)
        _pca_agree(got, ref, m)
        U, _, _ = opca.quantize(ref["Z"])
        assert np.array_equal(got["U"], U), trial


def test_representatives_random(host):
    rng = np.random.default_rng(22)
    for trial in range(20):
        n, d = int(rng.integers(1, 60)), int(rng.integers(2, 30))
        nc = int(rng.integers(1, 8))
        k = int(rng.integers(1, d + 1))
        Xq = rng.integers(0, 65536, (n, d)).astype(np.uint16)
        Xq[rng.random((n, d)) < 0.3] = 0
        labels = rng.integers(0, nc, n)
        for rep, fn in ((0, orep.mean_representatives), (1, orep.geomean_representatives)):
            assert host.representatives(Xq, labels, nc, k, rep) == fn(Xq, labels, nc, k), (trial, rep)


def test_tree_leaves_and_rules(host, table):
    T, P, tr, _ = table
    Xq = onorm.normalize(T[tr], onorm.STDCUT)
    shapes = [P[r] for r in tr]
    F = np.array(shapes, dtype=np.int64)
    for k in (4, 8):
        labels, nl = host.prune_tree_leaves(shapes, Xq, k)
        ref_labels, ref_nl = opt.leaf_labels(F, Xq, k)
        assert nl == ref_nl and np.array_equal(labels, ref_labels)
        assert host.representatives(Xq, labels, nl, k, 0) == host.prune_tree(shapes, Xq, k)
        assert host.representatives(Xq, labels, nl, k, 1) == \
            orep.geomean_representatives(Xq, ref_labels, ref_nl, k)


def test_evaluate_matches_the_regret_oracle(host, table):
    T, P, tr, te = table
    rng = np.random.default_rng(23)
    chosen = sorted(int(c) for c in rng.choice(T.shape[1], 8, replace=False))
    for rows in (te, tr, None):
        got = host.evaluate(T, rows=rows, chosen=chosen)
        ref = oreg.ceiling(T, chosen, rows)
        for key in ("geomean", "mean", "min", "frac_ge_0_9", "time_weighted"):
            assert abs(got[key] - ref[key]) <= 1e-12 * max(1.0, abs(ref[key])), key
        assert got["n"] == ref["n"]
    picks = [int(rng.integers(0, T.shape[1])) for _ in te]
    got = host.evaluate(T, rows=te, picks=picks)
    ref = oreg.selected(T, picks, te)
    for key in ("geomean", "mean", "min", "frac_ge_0_9", "time_weighted"):
        assert abs(got[key] - ref[key]) <= 1e-12 * max(1.0, abs(ref[key])), key


def test_evaluate_rejects_unmeasured(host, kt):
    T = np.array([[5, -1], [-1, -1]], dtype=np.int64)
    with pytest.raises(kt.KtError):
        host.evaluate(T, picks=[1, 0])
    with pytest.raises(kt.KtError):
        host.evaluate(T, rows=[1], chosen=[0])
    assert host.evaluate(T, rows=[0], chosen=[0, 1])["geomean"] == 1.0
