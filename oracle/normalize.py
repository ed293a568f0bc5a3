"""Normalization of one problem's performance vector (paper section 3.4,
"Normalization method").  Test infrastructure only.

The paper maps each problem's per-configuration performance into [0, 1] with
the best configuration at (or near) 1, in four ways:

* relative: performance divided by the best performance of that problem;
* raw cutoff: relative values below 0.9 are set to 0, others kept;
* standard cutoff: the raw cutoff followed by a rescale that uses the whole
  [0, 1] range;
* sigmoid: f(x) = 1 / (1 + exp(50 (0.85 - x))) of the relative value (the
  only equation of the section; f(0.85) = 0.5 and f(x) < 0.1 for x < 0.8).

Integer reading (so that CPU and GPU agree bit for bit): times are int64
nanoseconds; since the flop count is fixed within a problem, relative
performance is t_best / t.  Values are Q16 integers, 65535 = 1.0:

    q      = floor((2*65535*t_best + t) / (2*t))               (round half up)
    raw    = q if 10*q >= 9*65535 else 0
    std    = round_half_up((q - 58982) * 65535 / (65535 - 58982)) if kept else 0
             with 58982 = ceil(0.9*65535): [0.9, 1] is mapped linearly to [0, 1]
    sigmoid= LUT[q],  LUT[v] = floor(65535 / (1 + exp(50*(0.85 - v/65535))) + 0.5)

t_best is the minimum over the row's valid entries (t > 0); entries with
t <= 0 (not measured) map to 0.
"""
from __future__ import annotations

import math

import numpy as np

Q = 65535
STD_LO = 58982   # ceil(0.9 * 65535)

RELATIVE, RAWCUT, STDCUT, SIGMOID = 0, 1, 2, 3


def relative_row(t):
    t = [int(x) for x in t]
    valid = [x for x in t if x > 0]
    if not valid:
        return [0] * len(t)
    tb = min(valid)
    return [(2 * Q * tb + x) // (2 * x) if x > 0 else 0 for x in t]


def raw_cutoff(q: int) -> int:
    return q if 10 * q >= 9 * Q else 0


def std_cutoff(q: int) -> int:
    if 10 * q < 9 * Q:
        return 0
    num = (q - STD_LO) * Q
    den = Q - STD_LO
    return (2 * num + den) // (2 * den)


_LUT = None


def sigmoid_lut():
    global _LUT
    if _LUT is None:
        _LUT = [int(math.floor(Q / (1.0 + math.exp(50.0 * (0.85 - v / Q))) + 0.5))
                for v in range(Q + 1)]
    return _LUT


def normalize_row(t, method: int):
    q = relative_row(t)
    if method == RELATIVE:
        return q
    if method == RAWCUT:
        return [raw_cutoff(v) for v in q]
    if method == STDCUT:
        return [std_cutoff(v) for v in q]
    if method == SIGMOID:
        lut = sigmoid_lut()
        return [lut[v] for v in q]
    raise ValueError(method)


def normalize(T, method: int = RELATIVE) -> np.ndarray:
    """int64 time table [n_rows][n_configs] -> uint16 Q16 table."""
    T = np.asarray(T, dtype=np.int64)
    return np.array([normalize_row(row, method) for row in T], dtype=np.uint16).reshape(T.shape)
