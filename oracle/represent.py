"""From clusters to kernels (paper section 4.2, "Selecting the kernels to
deploy").  Test infrastructure only.

Section 4.2 gives two rules.  A clustering that yields a representative
point per cluster (a k-means centroid) deploys the configuration that
performs best for that representative.  A clustering that yields only
labels deploys, per cluster, the configuration that is best for the
geometric mean of the cluster's members.  Both are written out here on the
uint16 Q16 rows of the normalized table (65535 = 1.0).

Readings (the paper leaves these open):

* clusters are taken in label order 0..n_clusters-1; each picks its best
  configuration not already picked (lowest index on ties), so the picks are
  distinct, and picking stops once k are taken (a clustering with more
  clusters than k deploys its first k); an empty cluster picks nothing;
  when fewer than k picks result,
  the rest are the unpicked configurations with the largest column sums
  over all rows (of the values for the mean rule, of their logarithms for
  the geometric-mean rule), lowest index on ties;
* the "mean" rule scores a configuration by the rounded arithmetic mean
  floor((2 s + n) / (2 n)) of the members' values (s their sum): the
  centroid of the integer k-means;
* the "geometric mean" rule compares the members' products of values.  A
  normalized value of 0 (a cutoff normalization, or an unmeasured entry)
  counts as the smallest positive value, 1 / 65535, so every product is
  defined and a configuration that is poor anywhere loses to one that is
  fair everywhere.  Products are compared through a fixed-point logarithm:
  L[q] = round(2^32 * log2(max(q, 1) / 65535)) (FP64, round half to even),
  summed exactly in int64; the cluster size is common to every configuration
  of a cluster, so the largest sum is the largest geometric mean.
"""
from __future__ import annotations

import numpy as np

LOG_SCALE = 2 ** 32


def log2_table() -> np.ndarray:
    """L[q] for q = 0..65535 (int64)."""
    q = np.maximum(np.arange(65536, dtype=np.float64), 1.0)
    return np.rint(LOG_SCALE * np.log2(q / 65535.0)).astype(np.int64)


def pick_distinct(scores, k: int, fill_scores=None):
    """scores[c][j] (int) per cluster c (None for an empty cluster): the
    best unpicked j per cluster in order, then fill from fill_scores."""
    picked = []
    for sc in scores:
        if len(picked) == k:
            break
        if sc is None:
            continue
        order = sorted(range(len(sc)), key=lambda j: (-int(sc[j]), j))
        picked.append(next(j for j in order if j not in picked))
    if len(picked) < k and fill_scores is not None:
        for j in sorted(range(len(fill_scores)), key=lambda j: (-int(fill_scores[j]), j)):
            if len(picked) == k:
                break
            if j not in picked:
                picked.append(j)
    return picked[:k]


def _rounded_mean(rows: np.ndarray) -> np.ndarray:
    n = rows.shape[0]
    return (2 * rows.sum(axis=0) + n) // (2 * n)


def mean_representatives(Xq, labels, n_clusters: int, k: int):
    Xq = np.asarray(Xq, dtype=np.int64)
    labels = np.asarray(labels)
    scores = [(_rounded_mean(Xq[labels == c]) if np.any(labels == c) else None)
              for c in range(n_clusters)]
    return pick_distinct(scores, k, Xq.sum(axis=0))


def geomean_representatives(Xq, labels, n_clusters: int, k: int):
    L = log2_table()
    logs = L[np.asarray(Xq, dtype=np.int64)]
    labels = np.asarray(labels)
    scores = [(logs[labels == c].sum(axis=0) if np.any(labels == c) else None)
              for c in range(n_clusters)]
    return pick_distinct(scores, k, logs.sum(axis=0))
