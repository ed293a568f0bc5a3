"""Decision-tree selector of the library (host C++, no GPU needed) against the
CART oracle: node arrays and predictions must be identical bit for bit."""
import os

import numpy as np
import pytest

import synth
from oracle import cart

VARIANTS = {"A": 0, "B": 1, "C": 2}


def _table(rng, n_shapes, n_cfg, seed_shapes):
    shapes = [(m, n, k, b, ta, tb) for (m, n, k, b) in synth.sweep_shapes(n_shapes, seed_shapes)
              for (ta, tb) in synth.LAYOUTS]
    T = rng.integers(1000, 10 ** 7, size=(len(shapes), n_cfg)).astype(np.int64)
    # plant a structure so the tree has something to learn
    for i, (m, n, k, b, ta, tb) in enumerate(shapes):
        T[i, (m > 500) + 2 * (k > 300) + ta] //= 4
    return shapes, T


@pytest.mark.parametrize("variant", ["A", "B", "C"])
@pytest.mark.parametrize("k", [4, 8])
def test_tree_matches_oracle(kt, variant, k):
    rng = np.random.default_rng(100 + k)
    shapes, T = _table(rng, 120, 30, 777 + k)
    chosen = [int(c) for c in rng.choice(30, size=k, replace=False)]
    h = kt.Handle(-1)
    h.fit_selector(VARIANTS[variant], shapes, T, chosen)
    got = h.get_tree()
    y = cart.labels_from_times(T, chosen)
    X = np.array(shapes, dtype=np.int64)
    md, ml = cart.TREE_PARAMS[variant]
    ref = cart.fit(X, y, k, md, ml)
    assert got == {key: [int(v) for v in ref[key]] for key in ref}
    pred = cart.predict(ref, X)
    for i in range(0, len(shapes), 7):
        assert h.select(*shapes[i]) == chosen[pred[i]]


def test_tree_on_unseen_shapes(kt):
    rng = np.random.default_rng(5)
    shapes, T = _table(rng, 80, 20, 4242)
    chosen = [3, 9, 0, 17]
    h = kt.Handle(-1)
    h.fit_selector(1, shapes, T, chosen)
    ref = cart.fit(np.array(shapes), cart.labels_from_times(T, chosen), 4, 6, 3)
    for s in [(16, 16, 16, 1, 0, 0), (4096, 4096, 4096, 64, 1, 1), (700, 20, 5000, 3, 0, 1)]:
        assert h.select(*s) == chosen[cart.predict_one(ref, s)]


def test_save_load_roundtrip_and_corruption(kt, tmp_path):
    rng = np.random.default_rng(6)
    shapes, T = _table(rng, 60, 25, 99)
    chosen = [1, 2, 5]
    h = kt.Handle(-1)
    h.fit_selector(0, shapes, T, chosen)
    p = str(tmp_path / "sel.txt")
    h.save(p)
    h2 = kt.Handle(-1)
    h2.load(p)
    assert h2.get_tree() == h.get_tree()
    for s in shapes[::5]:
        assert h2.select(*s) == h.select(*s)
    txt = open(p).read()
    for bad in (txt.replace("KTSEL 3", "KTSEL 9"), txt[: len(txt) // 2], txt.replace("tree", "tre"),
                txt.replace("chosen 3 1 2 5", "chosen 3 1 2 999"), txt.replace("dtype 0", "dtype 7"),
                txt.replace("box 1 1", "box 2 1"), txt.replace("box 1 1", "box 1")):
        q = str(tmp_path / "bad.txt")
        open(q, "w").write(bad)
        h3 = kt.Handle(-1)
        with pytest.raises(kt.KtError) as e:
            h3.load(q)
        assert e.value.status == -6
    with pytest.raises(kt.KtError) as e:
        kt.Handle(-1).load(str(tmp_path / "missing.txt"))
    assert e.value.status == -6


def test_training_box_saved_and_version_2_files(kt, tmp_path):
    rng = np.random.default_rng(7)
    shapes, T = _table(rng, 40, 12, 5)
    h = kt.Handle(-1)
    h.fit_selector(1, shapes, T, [0, 4, 7])
    info = h.selector_info()
    S = np.array(shapes)
    assert info["kind"] == 1 and info["chosen"] == [0, 4, 7] and info["fallback"] == 1
    assert info["box_lo"] == S[:, :4].min(axis=0).tolist()
    assert info["box_hi"] == S[:, :4].max(axis=0).tolist()
    with pytest.raises(kt.KtError):
        h.set_fallback(3)
    h.set_fallback(2)
    h.fit_selector(2, shapes, T, [0, 4, 7])        # the setting survives a refit
    assert h.selector_info()["fallback"] == 2
    p = str(tmp_path / "sel.txt")
    h.save(p)
    h2 = kt.Handle(-1)
    h2.load(p)
    assert h2.selector_info() == h.selector_info()
    # a version 2 file (no box line) loads without a training box
    old = "".join(l for l in open(p) if not l.startswith("box")).replace("KTSEL 3", "KTSEL 2")
    q = str(tmp_path / "v2.txt")
    open(q, "w").write(old)
    h3 = kt.Handle(-1)
    h3.load(q)
    assert h3.selector_info()["box_hi"] == [-1] * 4
    assert all(h3.select(*s) == h.select(*s) for s in shapes[::3])


def test_select_before_fit(kt):
    h = kt.Handle(-1)
    with pytest.raises(kt.KtError) as e:
        h.select(64, 64, 64)
    assert e.value.status == -4


def test_bad_fit_arguments(kt):
    h = kt.Handle(-1)
    shapes = [(64, 64, 64, 1, 0, 0)] * 4
    T = np.ones((4, 10), np.int64)
    for chosen in ([1, 1], [10], [-1]):
        with pytest.raises(kt.KtError) as e:
            h.fit_selector(0, shapes, T, chosen)
        assert e.value.status == -1


def test_selectors_are_per_dtype(kt, tmp_path):
    """Each dtype has its own selector: fitting one leaves the others alone,
    and the file keeps all of them."""
    rng = np.random.default_rng(9)
    shapes, T = _table(rng, 50, 30, 123)
    h = kt.Handle(-1)
    h.fit_selector(0, shapes, T, [1, 2, 3], dtype=kt.F32)
    with pytest.raises(kt.KtError) as e:
        h.select(64, 64, 64, dtype=kt.BF16)
    assert e.value.status == -4
    T2 = T[:, ::-1].copy()
    h.fit_selector(2, shapes, T2, [10, 20], dtype=kt.BF16)
    assert all(h.select(*s, dtype=kt.F32) in (1, 2, 3) for s in shapes[::3])
    assert all(h.select(*s, dtype=kt.BF16) in (10, 20) for s in shapes[::3])
    ref = cart.fit(np.array(shapes), cart.labels_from_times(T2, [10, 20]), 2, 3, 4)
    assert h.get_tree(dtype=kt.BF16) == {key: [int(v) for v in ref[key]] for key in ref}
    p = str(tmp_path / "two.txt")
    h.save(p)
    h2 = kt.Handle(-1)
    h2.load(p)
    for s in shapes[::4]:
        assert h2.select(*s, dtype=kt.F32) == h.select(*s, dtype=kt.F32)
        assert h2.select(*s, dtype=kt.BF16) == h.select(*s, dtype=kt.BF16)
    with pytest.raises(kt.KtError):
        h2.select(64, 64, 64, dtype=kt.FP8E4M3)
    with pytest.raises(kt.KtError) as e:
        h.fit_selector(0, shapes, T, [98], dtype=kt.BF16)     # BF16 has 98 configurations
    assert e.value.status == -1
