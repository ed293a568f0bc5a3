"""Seeded input generators: pinned to published SplitMix64 outputs."""
import numpy as np

import synth


def test_splitmix64_published_vector():
    # Reference outputs of SplitMix64 seeded with 1234567 (Vigna's splitmix64.c).
    g = synth.SplitMix64(1234567)
    assert [g.next() for _ in range(5)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]


def test_counter_hash_matches_stream():
    # mix(s) is the first output of a stream whose state starts at s.
    for s in (0, 1, 12345, 2 ** 63 + 7):
        assert synth.mix64(s) == synth.SplitMix64(s).next()


def test_uniform_operand_exact_and_range():
    x = synth.uniform_operand(synth.operand_seed(1, 0), 100000)
    assert x.dtype == np.float32
    assert x.min() >= -1.0 and x.max() < 1.0
    # every value is a multiple of 2**-23: exact in FP32
    k = (x.astype(np.float64) + 1.0) * 2 ** 23
    assert np.array_equal(k, np.round(k))
    h = synth.mix64(synth.operand_seed(1, 0) ^ 7)
    assert x[7] == np.float32((h >> 40) * 2.0 ** -23 - 1.0)
    # offset addressing is the same stream
    assert np.array_equal(synth.uniform_operand(synth.operand_seed(1, 0), 10, offset=5), x[5:15])


def test_shape_sets():
    s = synth.sweep_shapes()
    assert len(s) == 300
    for (m, n, k, b) in s:
        assert 16 <= m <= 4096 and 16 <= n <= 4096 and 16 <= k <= 4096 and 1 <= b <= 64
    assert len(synth.sweep_problems()) == 1200
    tr, te = synth.train_test_split()
    assert len(tr) == 240 and len(te) == 60 and not set(tr) & set(te)
    g = synth.grouped_shapes()
    assert len(g) == 512 and all(32 <= v <= 2048 for sh in g for v in sh)
    c = synth.conv_shapes()
    assert len(c) == 156


def test_mlp_init_bounds():
    p = synth.mlp_init(8)
    assert p["W1"].shape == (64, 6) and p["W2"].shape == (64, 64) and p["W3"].shape == (8, 64)
    assert np.abs(p["W1"]).max() <= np.sqrt(6 / 6)
    assert np.abs(p["W2"]).max() <= np.sqrt(6 / 64)
    assert not p["b1"].any() and not p["b3"].any()
