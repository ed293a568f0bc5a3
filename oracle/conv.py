"""FP64 reference for the convolution layers that the selected GEMMs serve
(section 6 runs a VGG16-style network whose 3x3 convolutions, pooling and
fully connected layers are computed through matrix multiplications).  Test
infrastructure only: no product code imports this module.

Layout: activations NHWC (n, H, W, C); filters (R, S, Cin, Cout).  Every
function is the plain definition:

    y[b, i, j, o] = bias[o] + sum_{r, s, c} x[b, i*st - p + r, j*st - p + s, c] * w[r, s, c, o]

with out-of-range input positions reading 0 (zero padding), output size
(H + 2p - R) // st + 1, optional ReLU max(y, 0); 2x2 max pooling with stride 2
takes the largest of each disjoint 2x2 window (odd trailing rows / columns
dropped).  No transform (im2col, Winograd) appears here: both are ways of
reaching this same result.
"""
from __future__ import annotations

import numpy as np


def out_size(H, R, stride, pad):
    return (H + 2 * pad - R) // stride + 1


def conv2d(x, w, bias=None, stride=1, pad=1, relu=False):
    """Direct convolution in float64 (the definition above); one matrix
    product per filter tap."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n, H, W, C = x.shape
    R, S, C2, O = w.shape
    if C2 != C:
        raise ValueError("channel mismatch")
    Ho, Wo = out_size(H, R, stride, pad), out_size(W, S, stride, pad)
    xp = np.zeros((n, H + 2 * pad, W + 2 * pad, C))
    xp[:, pad:pad + H, pad:pad + W, :] = x
    y = np.zeros((n, Ho, Wo, O))
    for r in range(R):
        for s in range(S):
            win = xp[:, r:r + stride * (Ho - 1) + 1:stride, s:s + stride * (Wo - 1) + 1:stride, :]
            y += win @ w[r, s]
    if bias is not None:
        y += np.asarray(bias, dtype=np.float64)
    return np.maximum(y, 0.0) if relu else y


def conv2d_loops(x, w, bias=None, stride=1, pad=1, relu=False):
    """The same definition as nested scalar loops (small inputs only)."""
    n, H, W, C = x.shape
    R, S, _, O = w.shape
    Ho, Wo = out_size(H, R, stride, pad), out_size(W, S, stride, pad)
    y = np.zeros((n, Ho, Wo, O))
    for b in range(n):
        for i in range(Ho):
            for j in range(Wo):
                for o in range(O):
                    acc = 0.0 if bias is None else float(bias[o])
                    for r in range(R):
                        for s in range(S):
                            yi, xj = i * stride - pad + r, j * stride - pad + s
                            if 0 <= yi < H and 0 <= xj < W:
                                for c in range(C):
                                    acc += float(x[b, yi, xj, c]) * float(w[r, s, c, o])
                    y[b, i, j, o] = max(acc, 0.0) if relu else acc
    return y


def maxpool2x2(x):
    """2x2 max pooling, stride 2, on NHWC (odd trailing row / column dropped)."""
    x = np.asarray(x)
    n, H, W, C = x.shape
    Ho, Wo = H // 2, W // 2
    v = x[:, :2 * Ho, :2 * Wo, :].reshape(n, Ho, 2, Wo, 2, C)
    return v.max(axis=(2, 4))


# The VGG16 convolution stack (Simonyan and Zisserman, configuration D): 3x3
# convolutions, stride 1, padding 1, each followed by ReLU; "M" is a 2x2 max
# pool.  Then three fully connected layers 25088 -> 4096 -> 4096 -> 1000.
VGG16_LAYERS = [64, 64, "M", 128, 128, "M", 256, 256, 256, "M", 512, 512, 512, "M",
                512, 512, 512, "M"]
VGG16_FC = [(7 * 7 * 512, 4096), (4096, 4096), (4096, 1000)]
