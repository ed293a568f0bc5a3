"""Pins of the normalization oracle (section 3.4 of the paper)."""
import json
import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest

from oracle import normalize as nz

HERE = os.path.dirname(os.path.abspath(__file__))


def test_hand_computed_table():
    g = json.load(open(os.path.join(HERE, "golden", "normalize_3x3.json")))
    T = g["times"]
    assert nz.normalize(T, nz.RELATIVE).tolist() == g["relative"]
    assert nz.normalize(T, nz.RAWCUT).tolist() == g["rawcut"]
    assert nz.normalize(T, nz.STDCUT).tolist() == g["stdcut"]


def test_best_is_one_and_monotone():
    rng = np.random.default_rng(0)
    T = rng.integers(1000, 10 ** 9, size=(40, 57))
    for m in (nz.RELATIVE, nz.RAWCUT, nz.STDCUT, nz.SIGMOID):
        X = nz.normalize(T, m).astype(np.int64)
        for r in range(T.shape[0]):
            order = np.argsort(T[r], kind="stable")
            assert np.all(np.diff(X[r][order]) <= 0)          # slower never scores higher
        if m != nz.SIGMOID:
            assert np.all(X[np.arange(T.shape[0]), T.argmin(axis=1)] == 65535)


def test_relative_is_exact_ratio_rounded():
    # q is the integer nearest to 65535 * t_best / t (half up), checked with Fractions.
    from fractions import Fraction
    rng = np.random.default_rng(1)
    row = [int(v) for v in rng.integers(1, 10 ** 6, size=500)]
    tb = min(row)
    q = nz.relative_row(row)
    for t, v in zip(row, q):
        exact = Fraction(65535 * tb, t)
        assert v - Fraction(1, 2) <= exact < v + Fraction(1, 2)


def test_sigmoid_properties_from_paper():
    # The paper constructs f so that f(0.85) = 0.5 and f(x) < 0.1 for x < 0.8.
    lut = nz.sigmoid_lut()
    assert len(lut) == 65536
    assert all(a <= b for a, b in zip(lut, lut[1:]))
    q85 = round(0.85 * 65535)                 # 55705 (0.850004)
    assert lut[q85] == 32771                  # f(0.850004) * 65535 = 32770.6
    assert abs(lut[q85] - 32767.5) < 4
    q80 = math.floor(0.8 * 65535)             # 52428 <= 0.8
    assert lut[q80] == 4971 and lut[q80] < 6554   # 0.0759 < 0.1
    assert lut[65535] == 65499                # f(1) = 0.99945, not 1
    assert lut[0] == 0


def test_sigmoid_lut_against_decimal():
    # Independent evaluation in 40-digit decimal arithmetic.
    getcontext().prec = 40
    lut = nz.sigmoid_lut()
    for q in list(range(0, 65536, 97)) + [55705, 52428, 65535]:
        x = Decimal(q) / Decimal(65535)
        f = Decimal(65535) / (1 + (Decimal(50) * (Decimal("0.85") - x)).exp())
        assert lut[q] == int((f + Decimal("0.5")).to_integral_value(rounding="ROUND_FLOOR")), q


def test_cutoffs_boundary():
    assert nz.raw_cutoff(58981) == 0 and nz.raw_cutoff(58982) == 58982
    assert nz.std_cutoff(58981) == 0 and nz.std_cutoff(58982) == 0
    assert nz.std_cutoff(65535) == 65535
    # midpoint of [0.9, 1] maps to one half
    assert abs(nz.std_cutoff((58982 + 65535) // 2) - 32767) <= 6


def test_unmeasured_entries():
    assert nz.relative_row([-1, 5, 0, 10]) == [0, 65535, 0, 32768]
    assert nz.relative_row([-1, -1]) == [0, 0]
