"""Decision-tree selector (paper section 5.1, "Classifiers").
Test infrastructure only.

The paper labels every training problem with the chosen kernel that runs it
fastest and trains decision trees on the matrix sizes, in three variants:
A (no depth limit, leaves down to one sample), B (depth at most 6, at least
3 samples per leaf) and C (depth at most 3, at least 4 samples per leaf).
The tree is then emitted as nested if statements in the kernel launcher.

Integer CART reading (criterion, thresholds and ties are not stated):

* features are the raw integers (M, N, K, batch, transA, transB);
* Gini criterion: a split of n rows into L and R is scored by
  S = A/n_L + B/n_R with A = sum_c n_{L,c}^2, B = sum_c n_{R,c}^2 (maximising
  S minimises the weighted Gini impurity); scores are compared exactly by
  cross-multiplication;
* candidate thresholds lie between consecutive distinct values a < b of a
  feature at the node: t = floor(sqrt(a*b)) (a log-space midpoint,
  a <= t < b); a row goes left iff x <= t;
* features are scanned 0..5, thresholds ascending, and the first maximum wins;
* a node is split only if it is impure, depth < max_depth, both children keep
  >= min_leaf rows and the best S strictly exceeds the parent's sum_c n_c^2 / n;
* a leaf predicts its majority class (lowest class on ties);
* nodes are numbered in pre-order, left child first.

Labels: y = index j in ``chosen`` of the fastest chosen configuration (lowest j
on equal times).
"""
from __future__ import annotations

import math

import numpy as np

TREE_PARAMS = {"A": (None, 1), "B": (6, 3), "C": (3, 4)}   # (max_depth, min_leaf)


def labels_from_times(T, chosen):
    T = np.asarray(T, dtype=np.int64)
    sub = T[:, list(chosen)]
    # invalid (<=0) timings are never the fastest
    sub = np.where(sub > 0, sub, np.iinfo(np.int64).max)
    return np.argmin(sub, axis=1).astype(np.int64)


def _counts(y, n_classes):
    return np.bincount(y, minlength=n_classes).astype(object)


def fit(X, y, n_classes: int, max_depth, min_leaf: int):
    """Return the tree as a dict of lists: feature (-1 = leaf), threshold,
    left, right, cls."""
    X = np.asarray(X, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    feat, thr, left, right, cls = [], [], [], [], []

    def new_node():
        feat.append(-1); thr.append(0); left.append(-1); right.append(-1); cls.append(0)
        return len(feat) - 1

    def best_split(idx):
        n = len(idx)
        best = None   # (num, den, f, t)
        for f in range(X.shape[1]):
            order = sorted(idx, key=lambda i: X[i, f])
            vals = [int(X[i, f]) for i in order]
            cl = [0] * n_classes
            cr = [0] * n_classes
            for i in order:
                cr[y[i]] += 1
            pos = 0
            while pos < n:
                # move every row with the current value to the left side
                v = vals[pos]
                while pos < n and vals[pos] == v:
                    cl[y[order[pos]]] += 1
                    cr[y[order[pos]]] -= 1
                    pos += 1
                if pos == n:
                    break
                a, b = v, vals[pos]
                t = math.isqrt(a * b)
                nl, nr = pos, n - pos
                if nl < min_leaf or nr < min_leaf:
                    continue
                A = sum(c * c for c in cl)
                B = sum(c * c for c in cr)
                num, den = A * nr + B * nl, nl * nr
                if best is None or num * best[1] > best[0] * den:
                    best = (num, den, f, t)
        return best

    def build(idx, depth):
        node = new_node()
        cnt = [0] * n_classes
        for i in idx:
            cnt[y[i]] += 1
        cls[node] = max(range(n_classes), key=lambda c: (cnt[c], -c))
        n = len(idx)
        impure = sum(1 for c in cnt if c > 0) > 1
        if not impure or (max_depth is not None and depth >= max_depth) or n < 2 * min_leaf:
            return node
        sp = best_split(idx)
        if sp is None:
            return node
        num, den, f, t = sp
        P = sum(c * c for c in cnt)
        if not (num * n > P * den):
            return node
        feat[node], thr[node] = f, t
        li = [i for i in idx if X[i, f] <= t]
        ri = [i for i in idx if X[i, f] > t]
        left[node] = build(li, depth + 1)
        right[node] = build(ri, depth + 1)
        return node

    build(list(range(len(y))), 0)
    return dict(feature=feat, threshold=thr, left=left, right=right, cls=cls)


def predict_one(tree, x):
    node = 0
    while tree["feature"][node] >= 0:
        node = tree["left"][node] if x[tree["feature"][node]] <= tree["threshold"][node] \
            else tree["right"][node]
    return tree["cls"][node]


def predict(tree, X):
    return np.array([predict_one(tree, x) for x in np.asarray(X, dtype=np.int64)], dtype=np.int64)


def depth(tree, node=0):
    if tree["feature"][node] < 0:
        return 0
    return 1 + max(depth(tree, tree["left"][node]), depth(tree, tree["right"][node]))
