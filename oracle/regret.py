"""Evaluation of a kernel selection (paper section 4.3, "The results", and
section 5.1).  Test infrastructure only.

For each problem the achieved fraction of optimal performance is
r = t_best / t_used, with t_best the fastest time over all configurations of
that problem.  The ceiling of a pruned set uses the fastest chosen kernel;
a selector's value uses the kernel it picked.  Sets are summarised by the
geometric mean (the paper's figure), plus mean, minimum, the fraction of rows
at or above 0.9 and the time-weighted ratio sum(t_best) / sum(t_used).
"""
from __future__ import annotations

import math

import numpy as np


def _best(T):
    T = np.asarray(T, dtype=np.int64)
    return np.where(T > 0, T, np.iinfo(np.int64).max).min(axis=1)


def summary(r, t_best=None, t_used=None):
    r = np.asarray(r, dtype=np.float64)
    out = dict(geomean=float(math.exp(np.mean(np.log(r)))), mean=float(r.mean()),
               min=float(r.min()), frac_ge_0_9=float(np.mean(r >= 0.9)), n=int(r.size))
    if t_best is not None:
        out["time_weighted"] = float(np.sum(t_best) / np.sum(t_used))
    return out


def ceiling(T, chosen, rows=None):
    T = np.asarray(T, dtype=np.int64)
    rows = range(T.shape[0]) if rows is None else rows
    rows = list(rows)
    tb = _best(T)[rows]
    sub = T[np.ix_(rows, list(chosen))]
    tc = np.where(sub > 0, sub, np.iinfo(np.int64).max).min(axis=1)
    return summary(tb / tc, tb, tc)


def selected(T, picks, rows=None):
    """picks[i] = configuration index used for row rows[i]."""
    T = np.asarray(T, dtype=np.int64)
    rows = list(range(T.shape[0]) if rows is None else rows)
    tb = _best(T)[rows]
    ts = T[rows, list(picks)]
    return summary(tb / ts, tb, ts)
