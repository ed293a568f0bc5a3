"""GPU parity of the pruning variants against the oracle: k-means under the
normalization chosen on the training rows (kt_prune_auto), PCA + k-means
with both of section 4.2's cluster -> kernel rules (kt_prune_pca), and the
geometric-mean rule on k-means clusters and decision-tree leaves.  Every
step is integer or FP64 on the host, so picks, labels and inertia must
match bit for bit."""
import numpy as np
import pytest

import synth
from oracle import kmeans as okm
from oracle import normalize as onz
from oracle import pca as opca
from oracle import prune_tree as opt
from oracle import regret as oreg
from oracle import represent as orep

pytestmark = pytest.mark.gpu


def _draws(seed, n_init, k):
    return okm.restart_draws(synth.SplitMix64, seed, n_init, k)


def _planted(rng, n, d, groups):
    T = rng.integers(2000, 200000, size=(n, d)).astype(np.int64)
    fav = [rng.choice(d, size=3, replace=False) for _ in range(groups)]
    for i in range(n):
        T[i, fav[i % groups]] = rng.integers(900, 1100, size=3)
    return T


def _measured_train():
    from paper_2008_13145_amd import tune
    T, P, C, meta = tune.load_table(tune.DEFAULT_TABLE)
    rows = synth.rows_of_shapes(synth.train_test_split()[0])
    return T[rows], [tuple(int(v) for v in P[r]) for r in rows]


def _ws(kt, torch, n, d, k, n_init):
    b = kt.Handle.prune_workspace_bytes(n, d, k, n_init)
    return torch.empty(b, dtype=torch.uint8, device="cuda"), b


def test_prune_auto_matches_oracle(gpu, kt):
    h, torch = gpu
    rng = np.random.default_rng(31)
    n, d, k, n_init = 300, 48, 6, 4
    T = rng.integers(10_000, 2_000_000, size=(n, d)).astype(np.int64)
    T[: n // 2, :6] //= 5              # two regimes so the normalizations disagree
    T[n // 2:, 6:12] //= 3
    ws, wb = _ws(kt, torch, n, d, k, n_init)
    got = h.prune_auto(T, k, seed=13145, n_init=n_init, max_iter=100, workspace=ws, ws_bytes=wb)
    scores = []
    for norm in range(4):
        r = okm.kmeans(onz.normalize(T, norm), k, _draws(13145, n_init, k), 100)
        ch = okm.centroids_to_configs(r["centroids"])
        scores.append((oreg.ceiling(T, ch)["geomean"], ch))
        assert abs(got["scores"][norm] - scores[-1][0]) < 1e-12
    best = max(s for s, _ in scores)
    first = next(i for i, (s, _) in enumerate(scores) if s == best)
    assert got["norm"] == first and got["chosen"] == scores[first][1]


@pytest.mark.parametrize("source,norm,m,rep", [
    ("planted", 0, 8, opca.REP_CENTROID), ("planted", 2, 16, opca.REP_GEOMEAN),
    ("measured", 2, 16, opca.REP_CENTROID), ("measured", 2, 16, opca.REP_GEOMEAN),
    ("measured", 3, 8, opca.REP_CENTROID), ("measured", 1, 32, opca.REP_GEOMEAN)])
def test_prune_pca_bitwise(gpu, kt, source, norm, m, rep):
    h, torch = gpu
    if source == "planted":
        T = _planted(np.random.default_rng(m + norm), 960, 164, 9)
    else:
        T, _ = _measured_train()
    k, n_init, seed = 8, 10, 13145
    ws, wb = _ws(kt, torch, T.shape[0], T.shape[1], k, n_init)
    got = h.prune_pca(T, k, norm, m, rep=2 if rep == opca.REP_CENTROID else 1, seed=seed,
                      n_init=n_init, workspace=ws, ws_bytes=wb)
    ref = opca.prune_pca(T, k, norm, m, rep, _draws(seed, n_init, k))
    assert got["inertia"] == ref["inertia"]
    assert np.array_equal(got["labels"], ref["labels"])
    assert got["chosen"] == ref["chosen"]
    assert abs(got["explained"] - ref["explained"]) < 1e-12


@pytest.mark.parametrize("norm", [0, 2, 3])
def test_geomean_rule_on_kmeans_and_tree(gpu, kt, norm):
    from paper_2008_13145_amd import tune
    h, torch = gpu
    T, shapes = _measured_train()
    k = 8
    ws, wb = _ws(kt, torch, T.shape[0], T.shape[1], k, 10)
    Xq = onz.normalize(T, norm)
    got = tune.kmeans_pruning(h, T, k, 13145, norm, rep=1, workspace=ws, ws_bytes=wb)
    km = okm.kmeans(Xq, k, _draws(13145, 10, k), 300)
    assert got == orep.geomean_representatives(Xq, km["labels"], k, k)
    got_t = tune.tree_pruning(h, T, shapes, k, norm, rep=1)
    labels, nl = opt.leaf_labels(np.array(shapes, dtype=np.int64), Xq, k)
    assert got_t == orep.geomean_representatives(Xq, labels, nl, k)
