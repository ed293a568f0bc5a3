"""BF16 and FP8-e4m3 conversions used by the low-precision GEMM paths.
Test infrastructure only.

* BF16: round-to-nearest-even of the FP32 bit pattern,
  (u + 0x7FFF + ((u >> 16) & 1)) >> 16, with NaN kept quiet.
* FP8 e4m3 (OCP "e4m3fn": bias 7, no infinities, NaN = S.1111.111, largest
  finite 448): round to the nearest representable value, ties to the even
  code, saturating to +-448.
* Per-tensor FP8 scaling: s = 448 / amax (FP32 division, s = 1 if amax = 0);
  codes = e4m3(x * s) with the product rounded to FP32; dequantized value
  = decode(code) / s.
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def bf16_rne(x):
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    nan = np.isnan(np.asarray(x, dtype=np.float32))
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    r = np.where(nan, ((u >> 16) | 0x40).astype(np.uint16), r)
    return r


def bf16_decode(h):
    return (np.asarray(h, dtype=np.uint32) << 16).astype(np.uint32).view(np.float32)


def e4m3_decode_code(c: int) -> float:
    c = int(c) & 0xFF
    sign = -1.0 if c & 0x80 else 1.0
    e = (c >> 3) & 0xF
    m = c & 0x7
    if e == 0xF and m == 0x7:
        return float("nan")
    if e == 0:
        return sign * (m / 8.0) * 2.0 ** -6
    return sign * (1.0 + m / 8.0) * 2.0 ** (e - 7)


E4M3_TABLE = np.array([e4m3_decode_code(c) for c in range(256)], dtype=np.float64)
# positive finite codes 0x00..0x7E in increasing value order
_POS_VALS = E4M3_TABLE[:0x7F]


def e4m3_decode(codes):
    return E4M3_TABLE[np.asarray(codes, dtype=np.int64)]


def e4m3_encode(x):
    """Nearest e4m3 code, ties to even, saturating at +-448; NaN -> 0x7F."""
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    a = np.abs(x)
    sign = np.signbit(x)
    a_c = np.minimum(a, E4M3_MAX)
    hi = np.searchsorted(_POS_VALS, a_c, side="left")      # first value >= a
    hi = np.minimum(hi, 0x7E)
    lo = np.maximum(hi - 1, 0)
    vhi, vlo = _POS_VALS[hi], _POS_VALS[lo]
    dhi, dlo = vhi - a_c, a_c - vlo
    pick_hi = (dhi < dlo) | ((dhi == dlo) & ((hi & 1) == 0))
    code = np.where(a_c == vhi, hi, np.where(pick_hi, hi, lo)).astype(np.int64)
    code = np.where(sign, code | 0x80, code)
    code = np.where(np.isnan(x), 0x7F, code)
    return code.astype(np.uint8)


def fp8_scale(x) -> np.float32:
    amax = np.float32(np.max(np.abs(np.asarray(x, dtype=np.float32)))) if np.size(x) else np.float32(0)
    if amax == 0:
        return np.float32(1.0)
    return np.float32(np.float32(E4M3_MAX) / amax)


def quantize_fp8(x):
    x = np.asarray(x, dtype=np.float32)
    s = fp8_scale(x)
    y = (x * s).astype(np.float32)
    return e4m3_encode(y), s


def rel_frobenius(approx, exact) -> float:
    approx = np.asarray(approx, dtype=np.float64)
    exact = np.asarray(exact, dtype=np.float64)
    den = np.linalg.norm(exact)
    return float(np.linalg.norm(approx - exact) / den) if den > 0 else float(np.linalg.norm(approx))
