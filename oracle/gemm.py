"""FP64 reference GEMM (section 3 of the paper): ctypes front end of
``gemm_ref.c``.  Test infrastructure only.

``gemm(...)`` returns C_b = alpha*op(A_b)*op(B_b) + beta*C0_b as a dense
(batch, M, N) float64 array; ``gemm_sampled`` returns only chosen full rows and
full columns.  Arrays are flat float32 numpy buffers with the given leading
dimensions and batch strides (row-major; op() as in ``gemm_ref.c``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gemm_ref.c")
_LIB = os.path.join(_HERE, "_build", "liboracle_gemm.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile gemm_ref.c with gcc (OpenMP, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        os.makedirs(os.path.dirname(_LIB), exist_ok=True)
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i64, dbl, vp, ci = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_int
        lib.kt_oracle_gemm.argtypes = [i64, i64, i64, i64, ci, ci, dbl, dbl,
                                       vp, i64, i64, vp, i64, i64, vp, i64, i64, vp]
        lib.kt_oracle_gemm.restype = None
        lib.kt_oracle_gemm_sampled.argtypes = [i64, i64, i64, i64, ci, ci, dbl, dbl,
                                               vp, i64, i64, vp, i64, i64, vp, i64, i64,
                                               vp, i64, vp, i64, vp, vp]
        lib.kt_oracle_gemm_sampled.restype = None
        lib.kt_oracle_max_threads.restype = ci
        lib.kt_oracle_set_threads.argtypes = [ci]
        lib.kt_oracle_set_threads.restype = None
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().kt_oracle_max_threads())


def set_threads(n: int) -> None:
    """Threads of later oracle calls (timing only; results do not change)."""
    _load().kt_oracle_set_threads(int(n))


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f32(a):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float32).reshape(-1)
    return a


def gemm(M, N, K, batch, ta, tb, alpha, beta, A, lda, sA, B, ldb, sB, C0=None, ldc=0, sC=0):
    A, B, C0 = _f32(A), _f32(B), _f32(C0)
    if beta != 0 and C0 is None:
        raise ValueError("beta != 0 needs C0")
    out = np.empty((batch, M, N), dtype=np.float64)
    _load().kt_oracle_gemm(M, N, K, batch, ta, tb, float(alpha), float(beta),
                           _ptr(A), lda, sA, _ptr(B), ldb, sB,
                           _ptr(C0) if beta != 0 else None, ldc, sC, out.ctypes.data)
    return out


def gemm_sampled(M, N, K, batch, ta, tb, alpha, beta, A, lda, sA, B, ldb, sB,
                 C0, ldc, sC, rows, cols):
    A, B, C0 = _f32(A), _f32(B), _f32(C0)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out_r = np.empty((batch, len(rows), N), dtype=np.float64)
    out_c = np.empty((batch, M, len(cols)), dtype=np.float64)
    _load().kt_oracle_gemm_sampled(M, N, K, batch, ta, tb, float(alpha), float(beta),
                                   _ptr(A), lda, sA, _ptr(B), ldb, sB,
                                   _ptr(C0) if beta != 0 else None, ldc, sC,
                                   rows.ctypes.data, len(rows), cols.ctypes.data, len(cols),
                                   out_r.ctypes.data, out_c.ctypes.data)
    return out_r, out_c


def dense(a_op, b_op, alpha=1.0, beta=0.0, c0=None):
    """Convenience form on dense (batch, M, K) / (batch, K, N) float32 arrays
    given already in op() orientation (no transposes)."""
    a_op = np.asarray(a_op, dtype=np.float32)
    b_op = np.asarray(b_op, dtype=np.float32)
    if a_op.ndim == 2:
        a_op, b_op = a_op[None], b_op[None]
        c0 = None if c0 is None else np.asarray(c0)[None]
    bt, M, K = a_op.shape
    N = b_op.shape[2]
    return gemm(M, N, K, bt, 0, 0, alpha, beta, a_op, K, M * K, b_op, N, K * N,
                c0, N, M * N)
