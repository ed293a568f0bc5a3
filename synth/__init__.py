"""Seeded synthetic inputs shared by the oracle side and the library side.

This module holds no arithmetic of the method: only random streams, operand
values and problem-shape lists.  Both the CPU oracle (``oracle/``) and the GPU
library's tests and benchmark draw their inputs from here, so that the two
sides see identical data without sharing any code of the method itself.

Counter-based generator
-----------------------
Operands use SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) as a counter-based hash:

    mix(s)   = finalizer(s + 0x9E3779B97F4A7C15)
    x(seed, idx) = (mix(seed XOR idx) >> 40) * 2**-23 - 1      in [-1, 1)

The top 24 bits of the hash give a value that is exact in FP32.  The GPU fill
kernel implements the same published definition on its own; a test compares
the two bit for bit.

Shape sets
----------
``lu(rng, lo, hi, n) = clip(rint(exp(uniform(ln lo, ln hi, n))), lo, hi)``
(log-uniform integers), drawn in the order M, N, K, batch.

* ``sweep_shapes()``: 300 (M, N, K, batch) with M, N, K in 16..4096 and batch in
  1..64; this stands in for the 300 VGG/ResNet/MobileNet GEMM size sets of the
  paper's dataset (section 3, "A matrix multiply case study"), which is not
  available.  Each shape is used in all four transpose layouts.
* ``grouped_shapes()``: 512 (M, N, K) in 32..2048 for the grouped BF16 batch.
* ``conv_shapes()``: GEMMs of a VGG16-style 13-layer 3x3 conv stack at 224x224
  (section 6), lowered by im2col and by Winograd F(2x2,3x3).
"""
from __future__ import annotations

import math

import numpy as np

SEED = 13145
GOLDEN = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1

# ----------------------------------------------------------------------------
# SplitMix64
# ----------------------------------------------------------------------------


def _mix_np(s: np.ndarray) -> np.ndarray:
    """SplitMix64 output for state ``s`` (uint64 array); wraps mod 2**64."""
    with np.errstate(over="ignore"):
        z = s + np.uint64(GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def mix64(s: int) -> int:
    """Scalar SplitMix64 output for state ``s``."""
    z = (s + GOLDEN) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


class SplitMix64:
    """Sequential SplitMix64 stream: ``next()`` advances the state by the
    golden gamma and returns the finalized value."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        out = mix64(self.state)
        self.state = (self.state + GOLDEN) & MASK64
        return out

    def uniform(self) -> float:
        """Double in [0, 1) from the top 53 bits."""
        return (self.next() >> 11) * (1.0 / 9007199254740992.0)


def operand_seed(base: int, role: int) -> int:
    """Seed of one operand tensor: role 0 = A, 1 = B, 2 = C0, others free."""
    return mix64((base * 8 + role) & MASK64)


def _uniform_chunk(seed: int, offset: int, out: np.ndarray) -> None:
    idx = np.arange(offset, offset + out.size, dtype=np.uint64)
    h = _mix_np(np.uint64(seed & MASK64) ^ idx)
    u24 = (h >> np.uint64(40)).astype(np.int64)
    out[:] = u24.astype(np.float64) * (2.0 ** -23) - 1.0


def uniform_operand(seed: int, count: int, offset: int = 0, threads: int = 16) -> np.ndarray:
    """``count`` FP32 values x(seed, offset + i) in [-1, 1), as a flat array.
    Large requests are generated in chunks on a thread pool (numpy releases
    the GIL); every element depends only on (seed, index), so the result does
    not depend on the chunking."""
    out = np.empty(count, dtype=np.float32)
    chunk = 1 << 22
    if count <= chunk or threads <= 1:
        for c0 in range(0, count, chunk):
            _uniform_chunk(seed, offset + c0, out[c0:c0 + chunk])
        return out
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda c0: _uniform_chunk(seed, offset + c0, out[c0:c0 + chunk]),
                    range(0, count, chunk)))
    return out


# ----------------------------------------------------------------------------
# Shape sets
# ----------------------------------------------------------------------------


def lu(rng: np.random.Generator, lo: int, hi: int, n: int) -> np.ndarray:
    v = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), n)))
    return np.clip(v, lo, hi).astype(np.int64)


def sweep_shapes(n: int = 300, seed: int = SEED + 2):
    """List of (M, N, K, batch) for the configuration sweep."""
    rng = np.random.default_rng(seed)
    M = lu(rng, 16, 4096, n)
    N = lu(rng, 16, 4096, n)
    K = lu(rng, 16, 4096, n)
    B = lu(rng, 1, 64, n)
    return [(int(M[i]), int(N[i]), int(K[i]), int(B[i])) for i in range(n)]


LAYOUTS = ((0, 0), (0, 1), (1, 0), (1, 1))


def sweep_problems(n: int = 300, seed: int = SEED + 2):
    """All (M, N, K, batch, transA, transB): shape-major, layout-minor."""
    out = []
    for (m, nn, k, b) in sweep_shapes(n, seed):
        for (ta, tb) in LAYOUTS:
            out.append((m, nn, k, b, ta, tb))
    return out


def train_test_split(n_shapes: int = 300, n_train: int = 240, seed: int = SEED + 20):
    """Seeded permutation of shape indices -> (train shapes, test shapes),
    each sorted.  The split is by shape, so that the four layouts of one shape
    never straddle it."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n_shapes)
    return sorted(int(i) for i in perm[:n_train]), sorted(int(i) for i in perm[n_train:])


def train_validation_split(train_shapes, n_val: int = 48, seed: int = SEED + 21):
    """Seeded split of the training shapes into (fitting shapes, validation
    shapes), each sorted: the validation shapes choose between selectors
    without touching the test shapes."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(train_shapes))
    ids = [int(train_shapes[i]) for i in perm]
    return sorted(ids[n_val:]), sorted(ids[:n_val])


def shape_of_row(row: int, n_layouts: int = 4) -> int:
    return row // n_layouts


def rows_of_shapes(shape_ids, n_layouts: int = 4):
    return [s * n_layouts + l for s in shape_ids for l in range(n_layouts)]


def grouped_shapes(n: int = 512, seed: int = SEED + 4):
    """List of (M, N, K) for the grouped batch of uneven GEMMs."""
    rng = np.random.default_rng(seed)
    M = lu(rng, 32, 2048, n)
    N = lu(rng, 32, 2048, n)
    K = lu(rng, 32, 2048, n)
    return [(int(M[i]), int(N[i]), int(K[i])) for i in range(n)]


VGG_LAYERS = (
    (224, 3, 64), (224, 64, 64),
    (112, 64, 128), (112, 128, 128),
    (56, 128, 256), (56, 256, 256), (56, 256, 256),
    (28, 256, 512), (28, 512, 512), (28, 512, 512),
    (14, 512, 512), (14, 512, 512), (14, 512, 512),
)
VGG_BATCHES = (1, 2, 4, 8, 16, 32)


def conv_shapes():
    """GEMMs of a VGG16-style conv stack: list of dicts with keys
    layer, batch_images, lowering ('im2col' | 'winograd'), M, N, K, batch."""
    out = []
    for b in VGG_BATCHES:
        for li, (h, cin, cout) in enumerate(VGG_LAYERS):
            out.append(dict(layer=li, batch_images=b, lowering="im2col",
                            M=h * h * b, N=cout, K=9 * cin, batch=1))
            out.append(dict(layer=li, batch_images=b, lowering="winograd",
                            M=(h // 2) * (h // 2) * b, N=cout, K=cin, batch=16))
    return out


def mlp_init(k: int, seed: int = SEED + 5, n_in: int = 6, hidden: int = 64):
    """He-uniform initial weights U(+-sqrt(6/fan_in)) of a n_in->hidden->hidden->k
    network drawn from a SplitMix64 stream (W1, W2, W3 in that order, each
    row-major [fan_out][fan_in]); biases are zero.  Returned as float64 arrays;
    the GPU side receives the FP32 rounding of the same values."""
    rng = SplitMix64(seed)
    def mat(fan_out, fan_in):
        bound = math.sqrt(6.0 / fan_in)
        vals = [(2.0 * rng.uniform() - 1.0) * bound for _ in range(fan_out * fan_in)]
        return np.array(vals, dtype=np.float64).reshape(fan_out, fan_in)
    W1 = mat(hidden, n_in)
    W2 = mat(hidden, hidden)
    W3 = mat(k, hidden)
    return dict(W1=W1, b1=np.zeros(hidden), W2=W2, b2=np.zeros(hidden), W3=W3, b3=np.zeros(k))
