"""Decision-tree pruning of the configuration space (paper section 4.1,
"Decision tree": a regression tree from the matrix sizes to the performance
vector, limited to k leaves; each leaf's vector stands for the problems that
reach it and gives one kernel to deploy).  Test infrastructure only.

Integer reading (criterion, growth order, thresholds and ties are not
stated; the thresholds and the left/right rule follow the selector trees):

* features are the raw integers (M, N, K, batch, transA, transB); targets are
  the Q16 rows of the normalized table;
* a split of a node's n rows into L and R is scored by
  S = A / n_L + B / n_R with A = sum_j (sum_{i in L} x_ij)^2 and B likewise
  for R (maximising S minimises the summed squared error to the children's
  means); gain = S - P / n with P = sum_j (sum_i x_ij)^2; scores and gains are
  compared exactly as fractions;
* candidate thresholds lie between consecutive distinct values a < b of a
  feature at the node: t = floor(sqrt(a*b)); a row goes left iff x <= t;
  features are scanned 0..5, thresholds ascending, the first maximum wins;
* growth is best first: while there are fewer than k leaves, the leaf whose
  best split has the largest gain (earliest-created leaf on ties) is split,
  provided that gain is > 0; otherwise growth stops;
* leaves are taken in pre-order (left child first); each gives the
  configuration with the largest rounded mean floor((2 s + n) / (2 n)) of
  its rows (lowest index on ties), or its next best unchosen one, so the
  picks are distinct;
* with fewer than k leaves the remaining picks are the unchosen
  configurations with the largest column sums over all rows (lowest index on
  ties).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def _best_split(F, X, idx):
    """(gain as Fraction, feature, threshold) of the best split of rows idx,
    or None when every feature is constant on them."""
    n = len(idx)
    tot = X[idx].sum(axis=0)
    P = int((tot.astype(object) ** 2).sum())
    best = None
    for f in range(F.shape[1]):
        order = sorted(idx, key=lambda i: int(F[i, f]))
        vals = [int(F[i, f]) for i in order]
        left = np.zeros(X.shape[1], dtype=np.int64)
        pos = 0
        while pos < n:
            v = vals[pos]
            while pos < n and vals[pos] == v:
                left += X[order[pos]]
                pos += 1
            if pos == n:
                break
            t = math.isqrt(v * vals[pos])
            right = tot - left
            A = int((left.astype(object) ** 2).sum())
            B = int((right.astype(object) ** 2).sum())
            score = Fraction(A, pos) + Fraction(B, n - pos)
            if best is None or score > best[0]:
                best = (score, f, t)
    if best is None:
        return None
    return best[0] - Fraction(P, n), best[1], best[2]


def fit(F, X, k: int):
    """Grow the tree; returns (nodes, leaves_in_preorder) where nodes is a list
    of dicts {rows, feature, threshold, left, right}."""
    F = np.asarray(F, dtype=np.int64)
    X = np.asarray(X, dtype=np.int64)
    nodes = [dict(rows=list(range(len(X))), feature=-1, threshold=0, left=-1, right=-1)]
    leaves = [0]           # in creation order
    cand = {0: _best_split(F, X, nodes[0]["rows"])}
    while len(leaves) < k:
        pick = None
        for leaf in leaves:
            c = cand[leaf]
            if c is None or c[0] <= 0:
                continue
            if pick is None or c[0] > cand[pick][0]:
                pick = leaf
        if pick is None:
            break
        _, f, t = cand[pick]
        rows = nodes[pick]["rows"]
        li = [i for i in rows if F[i, f] <= t]
        ri = [i for i in rows if F[i, f] > t]
        nodes[pick].update(feature=f, threshold=t, left=len(nodes), right=len(nodes) + 1)
        for part in (li, ri):
            nodes.append(dict(rows=part, feature=-1, threshold=0, left=-1, right=-1))
            cand[len(nodes) - 1] = _best_split(F, X, part)
        leaves.remove(pick)
        leaves += [len(nodes) - 2, len(nodes) - 1]
    pre = []

    def walk(i):
        if nodes[i]["feature"] < 0:
            pre.append(i)
        else:
            walk(nodes[i]["left"])
            walk(nodes[i]["right"])
    walk(0)
    return nodes, pre


def leaf_labels(F, X, k: int):
    """(labels, n_leaves): the pre-order position of the leaf each row
    reaches, for the representative rules of ``oracle.represent``."""
    nodes, pre = fit(F, X, k)
    labels = np.zeros(len(X), dtype=np.int64)
    for pos, leaf in enumerate(pre):
        labels[nodes[leaf]["rows"]] = pos
    return labels, len(pre)


def prune(F, X, k: int):
    """The k configurations chosen by decision-tree pruning."""
    X = np.asarray(X, dtype=np.int64)
    nodes, pre = fit(F, X, k)
    chosen = []
    for leaf in pre:
        rows = nodes[leaf]["rows"]
        n = len(rows)
        m = (2 * X[rows].sum(axis=0) + n) // (2 * n)
        order = sorted(range(X.shape[1]), key=lambda j: (-int(m[j]), j))
        chosen.append(next(j for j in order if j not in chosen))
    col = X.sum(axis=0)
    for j in sorted(range(X.shape[1]), key=lambda j: (-int(col[j]), j)):
        if len(chosen) == k:
            break
        if j not in chosen:
            chosen.append(j)
    return chosen
