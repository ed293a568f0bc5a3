"""Pins of the convolution oracle against facts that do not come from its own
formula: brute-force scalar loops on tiny inputs, closed forms (the number of
in-bounds taps for constant data), an identity filter, a 1x1 filter that is a
plain matrix product, a library correlation on one channel, and a worked
pooling example."""
import numpy as np
import pytest
from scipy import signal

from oracle import conv as oc


@pytest.mark.parametrize("stride,pad,R", [(1, 1, 3), (2, 1, 3), (1, 0, 3), (2, 2, 5), (1, 0, 1)])
def test_matches_scalar_loops(stride, pad, R):
    rng = np.random.default_rng(R * 10 + stride + pad)
    x = rng.standard_normal((2, 7, 6, 3))
    w = rng.standard_normal((R, R, 3, 4))
    b = rng.standard_normal(4)
    for relu in (False, True):
        got = oc.conv2d(x, w, b, stride, pad, relu)
        ref = oc.conv2d_loops(x, w, b, stride, pad, relu)
        assert got.shape == ref.shape
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_constant_input_counts_in_bounds_taps():
    """All-ones input and filter, pad 1: each output is Cin times the number
    of the 3x3 taps that land inside the image (4 at corners, 6 on edges,
    9 inside)."""
    H, W, C = 5, 6, 3
    y = oc.conv2d(np.ones((1, H, W, C)), np.ones((3, 3, C, 2)))
    rows = np.array([2] + [3] * (H - 2) + [2])
    cols = np.array([2] + [3] * (W - 2) + [2])
    expect = C * np.outer(rows, cols)
    assert np.array_equal(y[0, :, :, 0], expect) and np.array_equal(y[0, :, :, 1], expect)


def test_identity_filter_returns_input():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 5, 4, 3))
    w = np.zeros((3, 3, 3, 3))
    w[1, 1] = np.eye(3)
    assert np.array_equal(oc.conv2d(x, w), x)


def test_one_by_one_filter_is_a_matrix_product():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, 4, 5, 6))
    w = rng.standard_normal((1, 1, 6, 7))
    ref = (x.reshape(-1, 6) @ w[0, 0]).reshape(3, 4, 5, 7)
    assert np.allclose(oc.conv2d(x, w, pad=0), ref, rtol=1e-13, atol=1e-13)


def test_single_channel_equals_library_correlation():
    """One input and one output channel: the definition is a 2-D
    cross-correlation with zero padding ('same' size for a 3x3 filter)."""
    rng = np.random.default_rng(3)
    img = rng.standard_normal((9, 11))
    k = rng.standard_normal((3, 3))
    ref = signal.correlate2d(img, k, mode="same", boundary="fill", fillvalue=0)
    got = oc.conv2d(img[None, :, :, None], k[:, :, None, None])[0, :, :, 0]
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_out_size():
    assert oc.out_size(224, 3, 1, 1) == 224
    assert oc.out_size(7, 3, 2, 1) == 4
    assert oc.out_size(5, 5, 2, 2) == 3


def test_maxpool_worked_example():
    x = np.array([[1, 5, 2, 0, 9],
                  [3, 4, 8, 1, 9],
                  [0, 0, 7, 6, 9]], dtype=np.float64)[None, :, :, None]
    assert np.array_equal(oc.maxpool2x2(x)[0, :, :, 0], np.array([[5, 8]]))
    x = np.full((1, 4, 4, 2), -3.0)
    assert np.array_equal(oc.maxpool2x2(x), np.full((1, 2, 2, 2), -3.0))


def test_vgg16_stack_shapes():
    """13 convolutions and 5 pools take 224x224x3 to 7x7x512 = 25088 features."""
    assert sum(1 for v in oc.VGG16_LAYERS if v != "M") == 13
    H, C = 224, 3
    for v in oc.VGG16_LAYERS:
        if v == "M":
            H //= 2
        else:
            C = v
    assert H * H * C == oc.VGG16_FC[0][0]
