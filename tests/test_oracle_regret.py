"""Pins of the evaluation oracle (section 4.3 of the paper)."""
import math

import numpy as np

from oracle import regret


def test_exhaustive_best_is_one():
    rng = np.random.default_rng(0)
    T = rng.integers(1, 1000, size=(50, 20))
    s = regret.selected(T, T.argmin(axis=1))
    assert s["geomean"] == 1.0 and s["min"] == 1.0 and s["time_weighted"] == 1.0


def test_ceiling_dominates_selector():
    rng = np.random.default_rng(1)
    T = rng.integers(1, 1000, size=(80, 30))
    chosen = [3, 7, 11]
    picks = rng.choice(chosen, size=80)
    c = regret.ceiling(T, chosen)
    s = regret.selected(T, picks)
    assert c["geomean"] >= s["geomean"] and c["min"] >= s["min"] and c["mean"] >= s["mean"]


def test_hand_computed():
    T = np.array([[10, 20, 40], [30, 15, 60], [8, 8, 4]])
    # chosen {0, 1}: best-of-chosen ratios 1, 1, 0.5 -> geomean 0.5**(1/3)
    c = regret.ceiling(T, [0, 1])
    assert math.isclose(c["geomean"], 0.5 ** (1 / 3))
    assert c["frac_ge_0_9"] == 2 / 3
    # picks (0, 0, 2): ratios 1, 0.5, 1
    s = regret.selected(T, [0, 0, 2])
    assert math.isclose(s["geomean"], 0.5 ** (1 / 3)) and s["min"] == 0.5
    assert math.isclose(s["time_weighted"], (10 + 15 + 4) / (10 + 30 + 4))
