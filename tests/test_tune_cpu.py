"""Host logic of the deploy tooling: the choice of normalization for the
k-means pruning (scored on the training rows by the geometric mean of
t_best / fastest chosen kernel), with the pruning itself taken from the
oracle through a stand-in handle."""
import numpy as np

import synth
from oracle import kmeans as okm
from oracle import normalize as onorm
from paper_2008_13145_amd import tune


class OraclePruner:
    """Stands in for a device handle: prune() runs the oracle k-means with the
    library's restart draws."""

    def __init__(self):
        self.calls = []

    def prune(self, T, k, norm, seed, n_init, max_iter, workspace=None, ws_bytes=0, stream=None):
        self.calls.append(norm)
        draws = okm.restart_draws(synth.SplitMix64, seed, n_init, k)
        r = okm.kmeans(onorm.normalize(np.asarray(T, np.int64), norm), k, draws, max_iter)
        return {"chosen": okm.centroids_to_configs(r["centroids"]), "inertia": int(r["inertia"])}


def _score(T, chosen):
    tb = T.min(axis=1).astype(np.float64)
    return float(np.exp(np.mean(np.log(tb / T[:, chosen].min(axis=1)))))


def test_select_pruning_picks_best_training_score():
    rng = np.random.default_rng(3)
    n, d = 90, 24
    T = rng.integers(10_000, 2_000_000, size=(n, d)).astype(np.int64)
    # two regimes so the normalizations disagree
    T[: n // 2, :6] //= 5
    T[n // 2:, 6:12] //= 3
    h = OraclePruner()
    res = tune.select_pruning(h, T, 4, 13145, n_init=3, max_iter=50)
    assert h.calls == [0, 1, 2, 3]
    scores = {}
    for norm, name in enumerate(tune.NORM_NAMES):
        chosen = OraclePruner().prune(T, 4, norm, 13145, 3, 50)["chosen"]
        scores[name] = _score(T, chosen)
        assert abs(res["train_ceiling"][name] - round(scores[name], 6)) < 1e-9
    best = max(scores.values())
    first_best = next(i for i, name in enumerate(tune.NORM_NAMES) if scores[name] == best)
    assert res["norm"] == first_best and res["norm_name"] == tune.NORM_NAMES[first_best]
    assert res["chosen"] == OraclePruner().prune(T, 4, first_best, 13145, 3, 50)["chosen"]


def test_select_pruning_ties_keep_the_earlier_normalization():
    class Same(OraclePruner):
        def prune(self, T, k, norm, seed, n_init, max_iter, **kw):
            return {"chosen": [0, 1], "inertia": 7}
    T = np.arange(1, 41, dtype=np.int64).reshape(10, 4) * 1000
    res = tune.select_pruning(Same(), T, 2, 1)
    assert res["norm"] == 0 and res["chosen"] == [0, 1]
    assert len(set(res["train_ceiling"].values())) == 1


def test_clusters_to_configs_matches_oracle_centroid_rule():
    """The reduced-space pruning's cluster -> configuration step equals the
    oracle's rounded-mean update followed by its centroid -> configuration
    rule, applied in the original normalized space."""
    rng = np.random.default_rng(11)
    for trial in range(5):
        n, d, k = 200, 30, 6
        Xq = rng.integers(0, 65536, size=(n, d)).astype(np.int64)
        labels = np.concatenate([np.arange(k), rng.integers(0, k, size=n - k)])
        rng.shuffle(labels)
        C = okm.update(Xq, labels, np.zeros(n, np.int64), np.zeros((k, d), np.int64))
        assert tune.clusters_to_configs(Xq, labels, k) == okm.centroids_to_configs(C)
