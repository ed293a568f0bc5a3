"""k-means pruning of the configuration space (paper section 4.1, "k-means
clustering", and section 4.2, "Selecting the kernels to deploy").
Test infrastructure only.

The paper clusters the normalized performance vectors of the training
problems (one point per problem, one coordinate per configuration) with
k-means -- k centroids that minimize the distance of every point to its
closest centroid -- and turns each centroid into one kernel to deploy by
taking the configuration that performs best for that representative.  The
baseline it compares against (Top-N) keeps the k configurations that are
best for the most problems.

The paper leaves initialisation, restarts, ties and rounding unstated; this
oracle fixes an all-integer reading so that any implementation can match it
exactly:

* points are the uint16 Q16 rows of the normalized table, distances are
  squared Euclidean in exact integers;
* initialisation is k-means++ (Arthur and Vassilvitskii, 2007), driven by a
  sequence of raw 64-bit draws passed in by the caller: the first centre is
  row ``draw mod n``; each later centre takes ``r = draw mod S`` with S the
  sum of every row's squared distance to its nearest chosen centre, and picks
  the first row whose running sum of those distances exceeds r (if S == 0:
  the lowest-index row not yet a centre);
* Lloyd iterations: assign each row to the nearest centroid (lowest index on
  ties); stop when the assignment repeats; otherwise move each centroid to the
  rounded mean floor((2*sum + n_j) / (2*n_j)) of its rows; a cluster left
  empty takes the row farthest from its assigned centroid (lowest index on
  ties), whose distance is then zeroed so the next empty cluster takes
  another row; after ``max_iter`` updates a final assignment is made;
* inertia is the sum of the final squared distances; of ``n_init`` restarts
  the lowest inertia wins (lowest restart on ties);
* centroid j -> the configuration with the largest centroid coordinate
  (lowest index on ties); if that configuration is already chosen, the
  centroid's next best unchosen one, so that exactly k distinct kernels
  result, in cluster order.
"""
from __future__ import annotations

import numpy as np


def sqdist_to(X: np.ndarray, c: np.ndarray) -> np.ndarray:
    d = X - c[None, :]
    return (d * d).sum(axis=1)


def kmeanspp_init(X: np.ndarray, k: int, draws) -> np.ndarray:
    """Indices of the k initial centres; ``draws`` yields raw 64-bit ints."""
    n = X.shape[0]
    draws = iter(draws)
    first = next(draws) % n
    centres = [first]
    D2 = sqdist_to(X, X[first])
    for _ in range(1, k):
        S = int(D2.sum())
        r = next(draws)
        if S == 0:
            pick = next(i for i in range(n) if i not in centres)
        else:
            r = r % S
            running = 0
            pick = None
            for i in range(n):
                running += int(D2[i])
                if running > r:
                    pick = i
                    break
        centres.append(pick)
        D2 = np.minimum(D2, sqdist_to(X, X[pick]))
    return np.array(centres, dtype=np.int64)


def assign(X: np.ndarray, C: np.ndarray):
    """Labels (lowest index among equal distances) and squared distances."""
    D = np.stack([sqdist_to(X, C[j]) for j in range(C.shape[0])], axis=1)
    labels = np.argmin(D, axis=1)          # argmin returns the first minimum
    return labels.astype(np.int64), D[np.arange(X.shape[0]), labels]


def update(X: np.ndarray, labels: np.ndarray, dist: np.ndarray, C: np.ndarray) -> np.ndarray:
    k = C.shape[0]
    newC = C.copy()
    dist = dist.copy()
    empty = []
    for j in range(k):
        members = X[labels == j]
        nj = members.shape[0]
        if nj == 0:
            empty.append(j)
            continue
        s = members.sum(axis=0)
        newC[j] = (2 * s + nj) // (2 * nj)
    for j in empty:
        far = int(np.argmax(dist))          # first maximum
        newC[j] = X[far]
        dist[far] = 0
    return newC


def lloyd(X: np.ndarray, init_idx: np.ndarray, max_iter: int):
    C = X[init_idx].copy()
    prev = None
    converged = False
    it = 0
    for it in range(max_iter):
        labels, dist = assign(X, C)
        if prev is not None and np.array_equal(labels, prev):
            converged = True
            break
        C = update(X, labels, dist, C)
        prev = labels
    if not converged:
        labels, dist = assign(X, C)
    return C, labels, int(dist.sum()), it


def kmeans(X, k: int, draws_per_restart, max_iter: int = 300):
    """Run len(draws_per_restart) restarts; return a dict with the winning
    centroids (int64 [k][d]), labels, inertia and restart index."""
    X = np.asarray(X, dtype=np.int64)
    if not (1 <= k <= X.shape[0]):
        raise ValueError("need 1 <= k <= n")
    best = None
    for r, draws in enumerate(draws_per_restart):
        init = kmeanspp_init(X, k, draws)
        C, labels, inertia, iters = lloyd(X, init, max_iter)
        if best is None or inertia < best["inertia"]:
            best = dict(centroids=C, labels=labels, inertia=inertia, restart=r,
                        init=init, iterations=iters)
    return best


def centroids_to_configs(C: np.ndarray):
    chosen = []
    for j in range(C.shape[0]):
        order = sorted(range(C.shape[1]), key=lambda f: (-int(C[j, f]), f))
        chosen.append(next(f for f in order if f not in chosen))
    return chosen


def top_n(Xq, k: int):
    """Top-N baseline (section 4.2): the k configurations that are best
    (largest normalized value, lowest index on ties) for the most rows;
    ties in the count go to the lower configuration index."""
    Xq = np.asarray(Xq, dtype=np.int64)
    best = np.argmax(Xq, axis=1)
    counts = np.bincount(best, minlength=Xq.shape[1])
    order = sorted(range(Xq.shape[1]), key=lambda f: (-int(counts[f]), f))
    return order[:k]


def restart_draws(gen_factory, seed: int, n_init: int, k: int):
    """Raw draws for each restart r: the first k outputs of the generator
    seeded with seed + r (mod 2**64).  ``gen_factory(seed)`` must return an
    object with ``next()``."""
    out = []
    for r in range(n_init):
        g = gen_factory((seed + r) & ((1 << 64) - 1))
        out.append([g.next() for _ in range(k)])
    return out
