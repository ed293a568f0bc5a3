"""kt: ML-pruned, per-shape-selected GEMM kernels for AMD MI355X (gfx950).

Thin ctypes binding of ``libkt.so`` (C ABI in ``include/kt.h``).  Every
function only marshals arguments; all work runs in the native library.  The
library must be built first (``python -m paper_2008_13145_amd.build``);
loading fails loudly otherwise -- there is no fallback implementation.

Device buffers are passed as integers (device addresses) or as objects with a
``data_ptr()`` method (e.g. torch tensors); streams as integers (hipStream_t)
or objects with a ``cuda_stream`` attribute.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("KT_LIBRARY", os.path.join(HERE, "libkt.so"))

F32, BF16, FP8E4M3 = 0, 1, 2
NORM_RELATIVE, NORM_RAWCUT, NORM_STDCUT, NORM_SIGMOID = 0, 1, 2, 3
REP_MEAN, REP_GEOMEAN, REP_CENTROID = 0, 1, 2
SEL_DT_A, SEL_DT_B, SEL_DT_C, SEL_MLP, SEL_EXHAUSTIVE = 0, 1, 2, 3, 4

STATUS = {0: "KT_OK", -1: "KT_EINVAL", -2: "KT_EUNSUPPORTED", -3: "KT_EHIP",
          -4: "KT_ENOTFITTED", -5: "KT_EWORKSPACE", -6: "KT_EIO"}

c_i32, c_i64, c_u64, c_f32, c_vp, c_sz = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                          ctypes.c_float, ctypes.c_void_p, ctypes.c_size_t)


class Shape(ctypes.Structure):
    _fields_ = [("M", c_i64), ("N", c_i64), ("K", c_i64), ("batch", c_i64),
                ("transA", c_i32), ("transB", c_i32)]


class Config(ctypes.Structure):
    _fields_ = [("bm", c_i32), ("bn", c_i32), ("t", c_i32), ("bk", c_i32), ("dtype", c_i32)]


class SweepOpts(ctypes.Structure):
    _fields_ = [("warmup", c_i32), ("target_ms", c_f32), ("min_reps", c_i32), ("max_reps", c_i32),
                ("cut_factor", c_f32), ("pause_ms", c_f32), ("seed", c_u64),
                ("alpha", c_f32), ("beta", c_f32), ("pad_rows", c_i32)]


class MlpOpts(ctypes.Structure):
    _fields_ = [("steps", c_i32), ("lr", c_f32), ("init", ctypes.POINTER(c_f32)), ("seed", c_u64),
                ("graph_steps", c_i32)]


class Eval(ctypes.Structure):
    _fields_ = [("geomean", ctypes.c_double), ("mean", ctypes.c_double), ("min", ctypes.c_double),
                ("frac_ge_0_9", ctypes.c_double), ("time_weighted", ctypes.c_double), ("n", c_i32)]


class GroupedOpts(ctypes.Structure):
    _fields_ = [("config_id", c_i32), ("small_config_id", c_i32), ("small_max_area", c_i64),
                ("schedule", c_i32), ("order", c_i32), ("wgs_per_cu", c_i32), ("pipeline", c_i32),
                ("visits", c_vp)]


class ConvShape(ctypes.Structure):
    _fields_ = [("n", c_i64), ("H", c_i64), ("W", c_i64), ("Cin", c_i64), ("Cout", c_i64),
                ("R", c_i32), ("S", c_i32), ("stride", c_i32), ("pad", c_i32)]


CONV_IM2COL, CONV_WINOGRAD, CONV_WINOGRAD_PRETRANSFORMED = 0, 1, 2


def conv_shape(n, H, W, Cin, Cout, R=3, S=3, stride=1, pad=1) -> ConvShape:
    return ConvShape(n, H, W, Cin, Cout, R, S, stride, pad)


class KtError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


_SIGS = {
    "kt_create": (c_i32, [ctypes.POINTER(c_vp), ctypes.c_int]),
    "kt_destroy": (c_i32, [c_vp]),
    "kt_last_error": (ctypes.c_char_p, [c_vp]),
    "kt_abi_version": (c_i32, []),
    "kt_num_configs": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_i32)]),
    "kt_get_config": (c_i32, [c_vp, c_i32, c_i32, ctypes.POINTER(Config)]),
    "kt_config_compiled": (c_i32, [c_vp, c_i32, c_i32, c_i32, c_i32, ctypes.POINTER(c_i32)]),
    "kt_gemm": (c_i32, [c_vp, c_i32, ctypes.POINTER(Shape), c_f32, c_vp, c_i64, c_i64, c_vp, c_i64,
                        c_i64, c_f32, c_vp, c_i64, c_i64, c_vp, c_vp, c_i32, c_vp]),
    "kt_gemm_splitk": (c_i32, [c_vp, c_i32, ctypes.POINTER(Shape), c_i32, c_f32, c_vp, c_i64,
                               c_i64, c_vp, c_i64, c_i64, c_f32, c_vp, c_i64, c_i64, c_vp, c_vp,
                               c_i32, c_vp, c_sz, c_vp, ctypes.POINTER(c_i32)]),
    "kt_gemm_splitk_workspace_bytes": (c_i32, [ctypes.POINTER(Shape), c_i32, ctypes.POINTER(c_sz)]),
    "kt_gemm_splitk_noalloc": (c_i32, [c_vp, c_i32, ctypes.POINTER(Shape), c_i32, c_f32, c_vp,
                                       c_i64, c_i64, c_vp, c_i64, c_i64, c_f32, c_vp, c_i64, c_i64,
                                       c_vp, c_vp, c_i32, c_vp, ctypes.POINTER(c_i32)]),
    "kt_gemm_splitk_noalloc_max_bytes": (c_i32, [ctypes.POINTER(c_sz)]),
    "kt_conv2d_gemm_shape": (c_i32, [ctypes.POINTER(ConvShape), c_i32, ctypes.POINTER(Shape)]),
    "kt_conv2d_workspace_bytes": (c_i32, [ctypes.POINTER(ConvShape), c_i32, c_i32,
                                          ctypes.POINTER(c_sz)]),
    "kt_conv2d": (c_i32, [c_vp, c_i32, ctypes.POINTER(ConvShape), c_vp, c_vp, c_vp, c_i32, c_vp,
                          c_i32, c_i32, c_vp, c_sz, c_vp]),
    "kt_winograd_filter": (c_i32, [c_vp, c_vp, c_i64, c_i64, c_vp, c_vp]),
    "kt_maxpool2x2": (c_i32, [c_vp, c_vp, c_i64, c_i64, c_i64, c_i64, c_vp, c_vp]),
    "kt_fill_uniform": (c_i32, [c_vp, c_vp, c_i64, c_u64, c_i64, c_vp]),
    "kt_convert_bf16": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_vp]),
    "kt_quantize_fp8": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "kt_num_kernels": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_i32)]),
    "kt_get_kernel": (c_i32, [c_vp, c_i32, c_i32, ctypes.POINTER(Config), ctypes.POINTER(c_i32),
                              ctypes.POINTER(c_i32)]),
    "kt_kernel_workspace_bytes": (c_i32, [c_vp, c_i32, ctypes.POINTER(Shape), c_i32,
                                          ctypes.POINTER(c_sz)]),
    "kt_set_workspace": (c_i32, [c_vp, c_vp, c_sz]),
    "kt_dma_pipeline": (c_i32, [c_vp, c_i32, ctypes.POINTER(Shape), c_vp, c_i64, c_i64, c_vp, c_i64,
                               c_i64, ctypes.POINTER(c_i32)]),
    "kt_set_full_rows": (c_i32, [c_vp, c_i32]),
    "kt_sweep_workspace_bytes": (c_i32, [ctypes.POINTER(Shape), c_i32, c_i32, ctypes.POINTER(c_sz)]),
    "kt_sweep": (c_i32, [c_vp, c_i32, ctypes.POINTER(Shape), c_i32, c_vp, c_i32,
                         ctypes.POINTER(SweepOpts), c_vp, c_sz, c_vp, c_vp]),
    "kt_normalize": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_i32, c_vp, c_vp]),
    "kt_prune_workspace_bytes": (c_i32, [c_i32, c_i32, c_i32, c_i32, ctypes.POINTER(c_sz)]),
    "kt_prune": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_i32, c_i32, c_u64, c_i32, c_i32, c_vp, c_sz,
                         c_vp, c_vp, ctypes.POINTER(c_i64), c_vp, c_vp]),
    "kt_prune_tree_leaves": (c_i32, [c_vp, ctypes.POINTER(Shape), c_vp, c_i32, c_i32, c_i32, c_vp,
                                     ctypes.POINTER(c_i32)]),
    "kt_representatives": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_vp, c_i32, c_i32, c_i32, c_vp]),
    "kt_log2_q16_table": (c_i32, [c_vp]),
    "kt_pca": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "kt_prune_pca": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_i32, c_u64, c_i32,
                             c_i32, c_vp, c_sz, c_vp, c_vp, ctypes.POINTER(c_i64), c_vp, c_vp]),
    "kt_prune_auto": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_i32, c_u64, c_i32, c_i32, c_vp, c_sz, c_vp,
                              c_vp, ctypes.POINTER(c_i32), c_vp]),
    "kt_evaluate": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_vp, c_i32, c_vp, c_vp, c_i32,
                            ctypes.POINTER(Eval)]),
    "kt_prune_topn": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_i32, c_vp, c_sz, c_vp, c_vp]),
    "kt_prune_tree": (c_i32, [c_vp, ctypes.POINTER(Shape), c_vp, c_i32, c_i32, c_i32, c_vp]),
    "kt_kmeans_u16": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_i32, c_u64, c_i32, c_i32, c_vp, c_sz,
                              c_vp, c_vp, c_vp, ctypes.POINTER(c_i64)]),
    "kt_fit_selector": (c_i32, [c_vp, c_i32, c_i32, ctypes.POINTER(Shape), c_vp, c_i32, c_i32, c_vp,
                                c_i32, ctypes.POINTER(MlpOpts), c_vp, c_sz, c_vp]),
    "kt_fit_selector_validated": (c_i32, [c_vp, c_i32, ctypes.POINTER(Shape), c_vp, c_i32, c_i32,
                                          c_vp, c_i32, c_vp, ctypes.POINTER(MlpOpts), c_vp, c_sz,
                                          c_vp, ctypes.POINTER(c_i32), c_vp]),
    "kt_set_fallback": (c_i32, [c_vp, c_i32, c_i32]),
    "kt_selector_info": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32), c_vp,
                                 c_vp, ctypes.POINTER(c_i32)]),
    "kt_select": (c_i32, [c_vp, c_i32, ctypes.POINTER(Shape), ctypes.POINTER(c_i32)]),
    "kt_select_batch": (c_i32, [c_vp, c_i32, c_vp, c_i32, c_vp, c_vp]),
    "kt_get_tree": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_i32), c_vp, c_vp, c_vp, c_vp, c_vp]),
    "kt_save": (c_i32, [c_vp, ctypes.c_char_p]),
    "kt_load": (c_i32, [c_vp, ctypes.c_char_p]),
    "kt_grouped_workspace_bytes": (c_i32, [ctypes.POINTER(Shape), c_i32, ctypes.POINTER(c_sz)]),
    "kt_grouped_num_candidates": (c_i32, [ctypes.POINTER(c_i32)]),
    "kt_grouped_plan_create": (c_i32, [c_vp, c_i32, ctypes.POINTER(Shape), c_i32, c_vp, c_vp, c_vp,
                                       c_vp, c_f32, c_f32, ctypes.POINTER(GroupedOpts), c_vp, c_sz,
                                       c_vp, ctypes.POINTER(c_vp)]),
    "kt_grouped_plan_launch": (c_i32, [c_vp, c_vp, c_vp]),
    "kt_grouped_plan_info": (c_i32, [c_vp, ctypes.POINTER(c_i32), ctypes.POINTER(GroupedOpts)]),
    "kt_grouped_plan_destroy": (c_i32, [c_vp]),
    "kt_grouped_gemm": (c_i32, [c_vp, c_i32, ctypes.POINTER(Shape), c_i32, c_vp, c_vp, c_vp, c_vp,
                                c_f32, c_f32, ctypes.POINTER(GroupedOpts), c_vp, c_sz, c_vp]),
    "kt_autotune_grouped": (c_i32, [c_vp, c_i32, ctypes.POINTER(Shape), c_i32, c_vp, c_vp, c_vp, c_vp,
                                    c_vp, c_sz, c_vp, ctypes.POINTER(GroupedOpts),
                                    ctypes.POINTER(c_f32), ctypes.POINTER(c_i32)]),
    "kt_mlp_workspace_bytes": (c_i32, [c_i32, c_i32, c_i32, ctypes.POINTER(c_sz)]),
    "kt_mlp_num_params": (c_i32, [c_i32, ctypes.POINTER(c_i32)]),
    "kt_mlp_features": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp]),
    "kt_mlp_forward_backward": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_i32, c_i32, c_vp, c_vp, c_vp,
                                        c_vp, c_sz, c_vp]),
    "kt_get_mlp": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_i32), c_vp]),
}

# Largest partial planes a split-K kernel takes from the kt_set_workspace
# buffer; a workspace this large lets every split-K kernel run split.
SPLIT_PLANE_CAP = 256 << 20

_lib = None


def lib(path: str | None = None):
    """Load libkt.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_2008_13145_amd.build` "
                           "(the GPU library has no fallback)")
    L = ctypes.CDLL(p)
    for name, (res, args) in _SIGS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = L
    return L


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take a pointer of {type(x)}")


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def shape(M, N, K, batch=1, transA=0, transB=0) -> Shape:
    return Shape(int(M), int(N), int(K), int(batch), int(transA), int(transB))


def shapes_array(rows):
    """Array of Shape from an iterable of (M, N, K, batch, transA, transB)."""
    rows = list(rows)
    arr = (Shape * max(1, len(rows)))()
    for i, r in enumerate(rows):
        arr[i] = shape(*r)
    return arr


class Handle:
    """One kt handle (``device=-1`` for a host-only handle)."""

    def __init__(self, device: int = 0, libpath: str | None = None):
        self.L = lib(libpath)
        h = c_vp()
        st = self.L.kt_create(ctypes.byref(h), int(device))
        if st != 0:
            raise KtError(st, self.L.kt_last_error(None).decode())
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            self.L.kt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise KtError(st, self.L.kt_last_error(self.h).decode())

    def status(self, st):
        """Return (status, message) without raising."""
        return st, (self.L.kt_last_error(self.h).decode() if st != 0 else "")

    # ------------------------------------------------------------ configs
    def num_configs(self, dtype=F32) -> int:
        n = c_i32()
        self._check(self.L.kt_num_configs(self.h, dtype, ctypes.byref(n)))
        return n.value

    def get_config(self, id, dtype=F32):
        c = Config()
        self._check(self.L.kt_get_config(self.h, dtype, int(id), ctypes.byref(c)))
        return (c.bm, c.bn, c.t, c.bk)

    def configs(self, dtype=F32):
        return [self.get_config(i, dtype) for i in range(self.num_configs(dtype))]

    def num_kernels(self, dtype=F32) -> int:
        n = c_i32()
        self._check(self.L.kt_num_kernels(self.h, dtype, ctypes.byref(n)))
        return n.value

    def get_kernel(self, id, dtype=F32):
        """(bm, bn, t, bk, slices) of kernel `id` and its base configuration id."""
        c, b, sl = Config(), c_i32(), c_i32()
        self._check(self.L.kt_get_kernel(self.h, dtype, int(id), ctypes.byref(c), ctypes.byref(b),
                                         ctypes.byref(sl)))
        return (c.bm, c.bn, c.t, c.bk, sl.value), b.value

    def kernels(self, dtype=F32):
        """(bm, bn, t, bk, slices) per kernel id: configurations, then split-K variants."""
        return [self.get_kernel(i, dtype)[0] for i in range(self.num_kernels(dtype))]

    def kernel_workspace_bytes(self, M, N, K, batch=1, transA=0, transB=0, id=0, dtype=F32) -> int:
        b = c_sz()
        self._check(self.L.kt_kernel_workspace_bytes(self.h, dtype,
                                                     ctypes.byref(shape(M, N, K, batch, transA, transB)),
                                                     int(id), ctypes.byref(b)))
        return b.value

    def dma_pipeline(self, dtype, shp: Shape, A, lda, sA, B, ldb, sB) -> bool:
        """True when BF16 / FP8 kernels run these operands through the LDS DMA pipeline."""
        v = c_i32()
        self._check(self.L.kt_dma_pipeline(self.h, int(dtype), ctypes.byref(shp), _ptr(A), int(lda),
                                          int(sA), _ptr(B), int(ldb), int(sB), ctypes.byref(v)))
        return bool(v.value)

    def set_full_rows(self, enabled: bool):
        """Promise that operands are allocated to whole rows of their leading dimension."""
        self._check(self.L.kt_set_full_rows(self.h, 1 if enabled else 0))

    def set_workspace(self, ws, ws_bytes=None):
        """Device buffer (tensor or pointer) kt_gemm gives split-K kernels; None clears it."""
        if ws is None:
            self._check(self.L.kt_set_workspace(self.h, None, 0))
            return
        n = ws_bytes if ws_bytes is not None else ws.numel() * ws.element_size()
        self._check(self.L.kt_set_workspace(self.h, _ptr(ws), int(n)))

    def config_compiled(self, id, transA, transB, dtype=F32) -> bool:
        v = c_i32()
        self._check(self.L.kt_config_compiled(self.h, dtype, int(id), int(transA), int(transB),
                                              ctypes.byref(v)))
        return bool(v.value)

    # --------------------------------------------------------------- gemm
    def gemm_raw(self, dtype, shp: Shape, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC,
                 scaleA=None, scaleB=None, config_id=-1, stream=None, check=True):
        st = self.L.kt_gemm(self.h, dtype, ctypes.byref(shp), float(alpha), _ptr(A), int(lda),
                            int(sA), _ptr(B), int(ldb), int(sB), float(beta), _ptr(C), int(ldc),
                            int(sC), _ptr(scaleA), _ptr(scaleB), int(config_id), _stream(stream))
        if check:
            self._check(st)
        return st

    @staticmethod
    def _operands(A, B, C, transA, transB):
        """(shape, lda, sA, ldb, sB, ldc, sC) of row-major device tensors."""
        def dims(t):
            # strides of size-1 dimensions carry no information and are ignored
            if t.dim() == 2:
                t = t.unsqueeze(0)
            b, r, c = t.shape
            if c > 1 and t.stride(2) != 1:
                raise ValueError("innermost dimension must be contiguous")
            ld = t.stride(1) if r > 1 else max(c, 1)
            st = t.stride(0) if b > 1 else r * ld
            return b, r, c, ld, st
        ba, ra, ca, lda, sA = dims(A)
        bb, rb, cb, ldb, sB = dims(B)
        bc, M, N, ldc, sC = dims(C)
        K = ra if transA else ca
        if (ca if transA else ra) != M or (rb if transB else cb) != N or (cb if transB else rb) != K:
            raise ValueError("inconsistent operand shapes")
        return shape(M, N, K, bc, transA, transB), lda, sA, ldb, sB, ldc, sC

    def gemm(self, A, B, C, transA=0, transB=0, alpha=1.0, beta=0.0, config_id=-1, dtype=F32,
             scaleA=None, scaleB=None, stream=None):
        """Batched GEMM on 3-D (or 2-D) row-major device tensors: A is
        (batch, M, K) or (batch, K, M) when transA, B is (batch, K, N) or
        (batch, N, K), C is (batch, M, N).  Leading dimensions and batch
        strides are read from the tensors' strides."""
        shp, lda, sA, ldb, sB, ldc, sC = self._operands(A, B, C, transA, transB)
        return self.gemm_raw(dtype, shp, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC,
                             scaleA, scaleB, config_id, stream)

    @staticmethod
    def splitk_workspace_bytes(M, N, K, batch, splits) -> int:
        b = c_sz()
        st = lib().kt_gemm_splitk_workspace_bytes(ctypes.byref(shape(M, N, K, batch)), int(splits),
                                                  ctypes.byref(b))
        if st != 0:
            raise KtError(st, "split-K workspace query")
        return b.value

    def gemm_splitk(self, A, B, C, splits, workspace, ws_bytes, transA=0, transB=0, alpha=1.0,
                    beta=0.0, config_id=-1, dtype=F32, scaleA=None, scaleB=None, stream=None):
        """Split-K GEMM on tensors laid out as for gemm(); returns the number
        of K slices used."""
        shp, lda, sA, ldb, sB, ldc, sC = self._operands(A, B, C, transA, transB)
        return self.gemm_splitk_raw(dtype, shp, splits, alpha, A, lda, sA, B, ldb, sB, beta, C,
                                    ldc, sC, workspace, ws_bytes, scaleA, scaleB, config_id,
                                    stream)

    def gemm_splitk_raw(self, dtype, shp: Shape, splits, alpha, A, lda, sA, B, ldb, sB, beta, C,
                        ldc, sC, workspace, ws_bytes, scaleA=None, scaleB=None, config_id=-1,
                        stream=None):
        used = c_i32(0)
        self._check(self.L.kt_gemm_splitk(self.h, dtype, ctypes.byref(shp), int(splits),
                                          float(alpha), _ptr(A), int(lda), int(sA), _ptr(B),
                                          int(ldb), int(sB), float(beta), _ptr(C), int(ldc),
                                          int(sC), _ptr(scaleA), _ptr(scaleB), int(config_id),
                                          _ptr(workspace), int(ws_bytes), _stream(stream),
                                          ctypes.byref(used)))
        return used.value

    @staticmethod
    def splitk_noalloc_max_bytes() -> int:
        b = c_sz()
        st = lib().kt_gemm_splitk_noalloc_max_bytes(ctypes.byref(b))
        if st != 0:
            raise KtError(st, "split-K scratch size query")
        return b.value

    def gemm_splitk_noalloc(self, A, B, C, splits, transA=0, transB=0, alpha=1.0, beta=0.0,
                            config_id=-1, dtype=F32, scaleA=None, scaleB=None, stream=None):
        """kt_gemm_splitk_noalloc on tensors laid out as for gemm() (partial
        planes in the library's static device scratch); returns the number of
        K slices used."""
        shp, lda, sA, ldb, sB, ldc, sC = self._operands(A, B, C, transA, transB)
        used = c_i32(0)
        self._check(self.L.kt_gemm_splitk_noalloc(self.h, dtype, ctypes.byref(shp), int(splits),
                                                  float(alpha), _ptr(A), int(lda), int(sA),
                                                  _ptr(B), int(ldb), int(sB), float(beta), _ptr(C),
                                                  int(ldc), int(sC), _ptr(scaleA), _ptr(scaleB),
                                                  int(config_id), _stream(stream),
                                                  ctypes.byref(used)))
        return used.value

    # -------------------------------------------------------- convolution
    @staticmethod
    def conv_gemm_shape(c: ConvShape, algo) -> tuple:
        out = Shape()
        st = lib().kt_conv2d_gemm_shape(ctypes.byref(c), int(algo), ctypes.byref(out))
        if st != 0:
            raise KtError(st, "conv GEMM shape query")
        return (out.M, out.N, out.K, out.batch, out.transA, out.transB)

    @staticmethod
    def conv_workspace_bytes(c: ConvShape, algo, splits=1) -> int:
        b = c_sz()
        st = lib().kt_conv2d_workspace_bytes(ctypes.byref(c), int(algo), int(splits),
                                             ctypes.byref(b))
        if st != 0:
            raise KtError(st, "conv workspace query")
        return b.value

    def conv2d(self, algo, c: ConvShape, x, w, bias, relu, y, workspace, ws_bytes, config_id=-1,
               splits=1, stream=None):
        self._check(self.L.kt_conv2d(self.h, int(algo), ctypes.byref(c), _ptr(x), _ptr(w),
                                     _ptr(bias), int(bool(relu)), _ptr(y), int(config_id),
                                     int(splits), _ptr(workspace), int(ws_bytes),
                                     _stream(stream)))

    def winograd_filter(self, w, Cin, Cout, U, stream=None):
        self._check(self.L.kt_winograd_filter(self.h, _ptr(w), int(Cin), int(Cout), _ptr(U),
                                              _stream(stream)))

    def maxpool2x2(self, x, n, H, W, C, y, stream=None):
        self._check(self.L.kt_maxpool2x2(self.h, _ptr(x), int(n), int(H), int(W), int(C), _ptr(y),
                                         _stream(stream)))

    def fill_uniform(self, dst, n, seed, offset=0, stream=None):
        self._check(self.L.kt_fill_uniform(self.h, _ptr(dst), int(n), int(seed) & (2 ** 64 - 1),
                                           int(offset), _stream(stream)))

    def convert_bf16(self, x, n, y, stream=None):
        self._check(self.L.kt_convert_bf16(self.h, _ptr(x), int(n), _ptr(y), _stream(stream)))

    def quantize_fp8(self, x, n, y, d_scale, workspace, ws_bytes=16, stream=None):
        self._check(self.L.kt_quantize_fp8(self.h, _ptr(x), int(n), _ptr(y), _ptr(d_scale),
                                           _ptr(workspace), int(ws_bytes), _stream(stream)))

    # -------------------------------------------------------------- sweep
    @staticmethod
    def sweep_workspace_bytes(shapes, dtype=F32) -> int:
        arr = shapes_array(shapes)
        b = c_sz()
        st = lib().kt_sweep_workspace_bytes(arr, len(shapes), dtype, ctypes.byref(b))
        if st != 0:
            raise KtError(st, "sweep workspace query")
        return b.value

    def sweep(self, shapes, workspace, ws_bytes, config_ids=None, time_ns=None, warmup=1,
              target_ms=2.0, min_reps=3, max_reps=200, cut_factor=8.0, pause_ms=0.0, seed=13145,
              alpha=1.0, beta=0.0, dtype=F32, stream=None, pad_rows=False):
        arr = shapes_array(shapes)
        n_cfg = self.num_kernels(dtype) if config_ids is None else len(config_ids)
        if time_ns is None:
            time_ns = np.full((len(shapes), n_cfg), -1, dtype=np.int64)
        assert time_ns.dtype == np.int64 and time_ns.flags.c_contiguous
        assert time_ns.shape == (len(shapes), n_cfg)
        ids = None
        if config_ids is not None:
            ids = np.ascontiguousarray(config_ids, dtype=np.int32)
        opts = SweepOpts(warmup, target_ms, min_reps, max_reps, cut_factor, pause_ms,
                         int(seed) & (2 ** 64 - 1), alpha, beta, 1 if pad_rows else 0)
        self._check(self.L.kt_sweep(self.h, dtype, arr, len(shapes),
                                    None if ids is None else ids.ctypes.data, n_cfg,
                                    ctypes.byref(opts), _ptr(workspace), int(ws_bytes),
                                    _stream(stream), time_ns.ctypes.data))
        return time_ns

    # -------------------------------------------------- normalize / prune
    def normalize(self, d_time, n_rows, n_configs, norm, d_out, stream=None):
        self._check(self.L.kt_normalize(self.h, _ptr(d_time), int(n_rows), int(n_configs), int(norm),
                                        _ptr(d_out), _stream(stream)))

    @staticmethod
    def prune_workspace_bytes(n_rows, n_configs, k, n_init) -> int:
        b = c_sz()
        st = lib().kt_prune_workspace_bytes(n_rows, n_configs, k, n_init, ctypes.byref(b))
        if st != 0:
            raise KtError(st, "prune workspace query")
        return b.value

    def prune(self, time_ns, k, norm=NORM_RELATIVE, seed=13145, n_init=10, max_iter=300,
              workspace=None, ws_bytes=0, stream=None):
        T = np.ascontiguousarray(time_ns, dtype=np.int64)
        n, d = T.shape
        chosen = np.zeros(k, dtype=np.int32)
        labels = np.zeros(n, dtype=np.int32)
        cents = np.zeros((k, d), dtype=np.int64)
        inertia = c_i64()
        self._check(self.L.kt_prune(self.h, T.ctypes.data, n, d, int(k), int(norm),
                                    int(seed) & (2 ** 64 - 1), int(n_init), int(max_iter),
                                    _ptr(workspace), int(ws_bytes), _stream(stream),
                                    chosen.ctypes.data, ctypes.byref(inertia), labels.ctypes.data,
                                    cents.ctypes.data))
        return dict(chosen=chosen.tolist(), inertia=inertia.value, labels=labels, centroids=cents)

    def prune_topn(self, time_ns, k, workspace=None, ws_bytes=0, stream=None):
        T = np.ascontiguousarray(time_ns, dtype=np.int64)
        chosen = np.zeros(k, dtype=np.int32)
        self._check(self.L.kt_prune_topn(self.h, T.ctypes.data, T.shape[0], T.shape[1], int(k),
                                         _ptr(workspace), int(ws_bytes), _stream(stream),
                                         chosen.ctypes.data))
        return chosen.tolist()

    def prune_tree(self, shapes, Xq, k):
        """Decision-tree pruning of the normalized Q16 table Xq (n x d host
        array, e.g. from normalize()) over the problem shapes; returns the k
        chosen configuration ids."""
        Xq = np.ascontiguousarray(np.asarray(Xq).astype(np.uint16))
        n, d = Xq.shape
        arr = shapes_array(shapes)
        out = np.zeros(k, dtype=np.int32)
        self._check(self.L.kt_prune_tree(self.h, arr, Xq.ctypes.data, n, d, int(k), out.ctypes.data))
        return [int(v) for v in out]

    def prune_tree_leaves(self, shapes, Xq, k):
        """Leaf (pre-order position) of every row under decision-tree pruning;
        returns (labels, n_leaves)."""
        Xq = np.ascontiguousarray(np.asarray(Xq).astype(np.uint16))
        n, d = Xq.shape
        labels = np.zeros(n, dtype=np.int32)
        nl = c_i32()
        self._check(self.L.kt_prune_tree_leaves(self.h, shapes_array(shapes), Xq.ctypes.data, n, d,
                                                int(k), labels.ctypes.data, ctypes.byref(nl)))
        return labels, nl.value

    def representatives(self, Xq, labels, n_clusters, k, rep=REP_MEAN):
        """One configuration per cluster (section 4.2) from labels on a Q16 table."""
        Xq = np.ascontiguousarray(np.asarray(Xq).astype(np.uint16))
        lab = np.ascontiguousarray(labels, dtype=np.int32)
        out = np.zeros(k, dtype=np.int32)
        self._check(self.L.kt_representatives(self.h, Xq.ctypes.data, Xq.shape[0], Xq.shape[1],
                                              lab.ctypes.data, int(n_clusters), int(k), int(rep),
                                              out.ctypes.data))
        return [int(v) for v in out]

    @staticmethod
    def log2_q16_table():
        t = np.zeros(65536, dtype=np.int64)
        st = lib().kt_log2_q16_table(t.ctypes.data)
        if st != 0:
            raise KtError(st, "log table")
        return t

    def pca(self, Xq, m):
        """Principal components of a Q16 table: dict(mean, components,
        variances, U, lo, span, explained)."""
        Xq = np.ascontiguousarray(np.asarray(Xq).astype(np.uint16))
        n, d = Xq.shape
        mean = np.zeros(d)
        comps = np.zeros((m, d))
        var = np.zeros(d)
        U = np.zeros((n, m), dtype=np.uint16)
        ls = np.zeros(2)
        ex = ctypes.c_double()
        self._check(self.L.kt_pca(self.h, Xq.ctypes.data, n, d, int(m), mean.ctypes.data,
                                  comps.ctypes.data, var.ctypes.data, U.ctypes.data, ls.ctypes.data,
                                  ctypes.byref(ex)))
        return dict(mean=mean, components=comps, variances=var, U=U, lo=float(ls[0]),
                    span=float(ls[1]), explained=ex.value)

    def prune_pca(self, time_ns, k, norm, m, rep=REP_CENTROID, seed=13145, n_init=10,
                  max_iter=300, workspace=None, ws_bytes=0, stream=None):
        T = np.ascontiguousarray(time_ns, dtype=np.int64)
        n, d = T.shape
        chosen = np.zeros(k, dtype=np.int32)
        labels = np.zeros(n, dtype=np.int32)
        inertia = c_i64()
        ex = ctypes.c_double()
        self._check(self.L.kt_prune_pca(self.h, T.ctypes.data, n, d, int(k), int(norm), int(m),
                                        int(rep), int(seed) & (2 ** 64 - 1), int(n_init),
                                        int(max_iter), _ptr(workspace), int(ws_bytes),
                                        _stream(stream), chosen.ctypes.data, ctypes.byref(inertia),
                                        labels.ctypes.data, ctypes.byref(ex)))
        return dict(chosen=[int(c) for c in chosen], labels=labels, inertia=inertia.value,
                    explained=ex.value)

    def prune_auto(self, time_ns, k, seed=13145, n_init=10, max_iter=300, workspace=None,
                   ws_bytes=0, stream=None):
        """k-means pruning under the normalization whose chosen set keeps the
        most of the optimum on these rows: dict(chosen, norm, scores)."""
        T = np.ascontiguousarray(time_ns, dtype=np.int64)
        n, d = T.shape
        chosen = np.zeros(k, dtype=np.int32)
        norm = c_i32()
        scores = np.zeros(4)
        self._check(self.L.kt_prune_auto(self.h, T.ctypes.data, n, d, int(k),
                                         int(seed) & (2 ** 64 - 1), int(n_init), int(max_iter),
                                         _ptr(workspace), int(ws_bytes), _stream(stream),
                                         chosen.ctypes.data, ctypes.byref(norm), scores.ctypes.data))
        return dict(chosen=[int(c) for c in chosen], norm=norm.value, scores=scores.tolist())

    def evaluate(self, time_ns, rows=None, picks=None, chosen=None):
        """Fraction-of-optimal summary (section 4.3): a selector's picks per
        evaluated row, or the ceiling of a chosen set; returns a dict."""
        T = np.ascontiguousarray(time_ns, dtype=np.int64)
        r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
        p = None if picks is None else np.ascontiguousarray(picks, dtype=np.int32)
        c = None if chosen is None else np.ascontiguousarray(chosen, dtype=np.int32)
        out = Eval()
        self._check(self.L.kt_evaluate(self.h, T.ctypes.data, T.shape[0], T.shape[1],
                                       None if r is None else r.ctypes.data,
                                       0 if r is None else len(r),
                                       None if p is None else p.ctypes.data,
                                       None if c is None else c.ctypes.data,
                                       0 if c is None else len(c), ctypes.byref(out)))
        return dict(geomean=out.geomean, mean=out.mean, min=out.min, frac_ge_0_9=out.frac_ge_0_9,
                    time_weighted=out.time_weighted, n=out.n)

    def kmeans_u16(self, X, k, seed=13145, n_init=10, max_iter=300, workspace=None, ws_bytes=0,
                   stream=None):
        """k-means on arbitrary 16-bit vectors (host array n x d)."""
        Xa = np.ascontiguousarray(X, dtype=np.uint16)
        n, d = Xa.shape
        labels = np.zeros(n, dtype=np.int32)
        cent = np.zeros((k, d), dtype=np.int64)
        inertia = c_i64()
        self._check(self.L.kt_kmeans_u16(self.h, Xa.ctypes.data, n, d, int(k), int(seed),
                                         int(n_init), int(max_iter), _ptr(workspace),
                                         int(ws_bytes), _stream(stream), labels.ctypes.data,
                                         cent.ctypes.data, ctypes.byref(inertia)))
        return {"labels": labels, "centroids": cent, "inertia": inertia.value}

    # ------------------------------------------------------------- select
    def fit_selector(self, kind, shapes, time_ns, chosen, mlp_steps=3000, mlp_lr=1e-3,
                     mlp_init=None, mlp_seed=13150, mlp_graph_steps=25, workspace=None, ws_bytes=0,
                     stream=None, dtype=F32):
        arr = shapes_array(shapes)
        T = np.ascontiguousarray(time_ns, dtype=np.int64)
        ch = np.ascontiguousarray(chosen, dtype=np.int32)
        opts = None
        keep = None
        if kind == SEL_MLP:
            init_ptr = None
            if mlp_init is not None:
                keep = np.ascontiguousarray(mlp_init, dtype=np.float32)
                init_ptr = keep.ctypes.data_as(ctypes.POINTER(c_f32))
            opts = MlpOpts(int(mlp_steps), float(mlp_lr), init_ptr, int(mlp_seed), int(mlp_graph_steps))
        self._check(self.L.kt_fit_selector(self.h, int(dtype), int(kind), arr, T.ctypes.data, T.shape[0],
                                           T.shape[1], ch.ctypes.data, len(ch),
                                           None if opts is None else ctypes.byref(opts),
                                           _ptr(workspace), int(ws_bytes), _stream(stream)))
        del keep

    def fit_selector_validated(self, shapes, time_ns, chosen, is_validation, mlp_steps=3000,
                               mlp_lr=1e-3, mlp_seed=13150, mlp_graph_steps=25, workspace=None,
                               ws_bytes=0, stream=None, dtype=F32):
        """Fit trees A/B/C and the MLP on the non-validation rows, keep the
        kind that scores best on the validation rows, refit it on all rows.
        Returns (kind, [score per kind])."""
        arr = shapes_array(shapes)
        T = np.ascontiguousarray(time_ns, dtype=np.int64)
        ch = np.ascontiguousarray(chosen, dtype=np.int32)
        val = np.ascontiguousarray(np.asarray(is_validation, dtype=bool).astype(np.uint8))
        assert len(val) == T.shape[0]
        opts = MlpOpts(int(mlp_steps), float(mlp_lr), None, int(mlp_seed), int(mlp_graph_steps))
        kind = c_i32()
        scores = np.zeros(4)
        self._check(self.L.kt_fit_selector_validated(
            self.h, int(dtype), arr, T.ctypes.data, T.shape[0], T.shape[1], ch.ctypes.data, len(ch),
            val.ctypes.data, ctypes.byref(opts), _ptr(workspace), int(ws_bytes), _stream(stream),
            ctypes.byref(kind), scores.ctypes.data))
        return kind.value, scores.tolist()

    def set_fallback(self, mode, dtype=F32):
        """0 off, 1 (True) the deployed kernels, 2 exhaustive over the library."""
        self._check(self.L.kt_set_fallback(self.h, int(dtype), int(mode)))

    def selector_info(self, dtype=F32):
        kind, k, fb = c_i32(), c_i32(), c_i32()
        self._check(self.L.kt_selector_info(self.h, int(dtype), ctypes.byref(kind), ctypes.byref(k),
                                            None, None, None))
        ch = np.zeros(max(k.value, 1), dtype=np.int32)
        box = np.zeros(8, dtype=np.int64)
        self._check(self.L.kt_selector_info(self.h, int(dtype), ctypes.byref(kind), ctypes.byref(k),
                                            ch.ctypes.data, box.ctypes.data, ctypes.byref(fb)))
        return dict(kind=kind.value, chosen=ch[:k.value].tolist(), box_lo=box[:4].tolist(),
                    box_hi=box[4:].tolist(), fallback=fb.value)

    def select(self, M, N, K, batch=1, transA=0, transB=0, dtype=F32) -> int:
        v = c_i32()
        s = shape(M, N, K, batch, transA, transB)
        self._check(self.L.kt_select(self.h, int(dtype), ctypes.byref(s), ctypes.byref(v)))
        return v.value

    def select_batch(self, d_shapes, n, d_ids, stream=None, dtype=F32):
        self._check(self.L.kt_select_batch(self.h, int(dtype), _ptr(d_shapes), int(n), _ptr(d_ids),
                                           _stream(stream)))

    def get_tree(self, dtype=F32):
        n = c_i32()
        self._check(self.L.kt_get_tree(self.h, int(dtype), ctypes.byref(n), None, None, None, None,
                                       None))
        f = np.zeros(n.value, np.int32)
        t = np.zeros(n.value, np.int64)
        l = np.zeros(n.value, np.int32)
        r = np.zeros(n.value, np.int32)
        c = np.zeros(n.value, np.int32)
        self._check(self.L.kt_get_tree(self.h, int(dtype), ctypes.byref(n), f.ctypes.data,
                                       t.ctypes.data, l.ctypes.data, r.ctypes.data, c.ctypes.data))
        return dict(feature=f.tolist(), threshold=t.tolist(), left=l.tolist(), right=r.tolist(),
                    cls=c.tolist())

    def save(self, path):
        self._check(self.L.kt_save(self.h, path.encode()))

    def load(self, path):
        self._check(self.L.kt_load(self.h, path.encode()))

    # ---------------------------------------------------------------- mlp
    @staticmethod
    def mlp_workspace_bytes(n_rows, n_configs, k) -> int:
        b = c_sz()
        st = lib().kt_mlp_workspace_bytes(n_rows, n_configs, k, ctypes.byref(b))
        if st != 0:
            raise KtError(st, "MLP workspace query")
        return b.value

    @staticmethod
    def mlp_num_params(k) -> int:
        v = c_i32()
        st = lib().kt_mlp_num_params(k, ctypes.byref(v))
        if st != 0:
            raise KtError(st, "MLP parameter count")
        return v.value

    def mlp_features(self, d_shapes, n, d_X, stream=None):
        self._check(self.L.kt_mlp_features(self.h, _ptr(d_shapes), int(n), _ptr(d_X), _stream(stream)))

    def mlp_forward_backward(self, d_params, d_X, d_Y, n, k, d_pred=None, d_grad=None, d_loss=None,
                             workspace=None, ws_bytes=0, stream=None):
        self._check(self.L.kt_mlp_forward_backward(self.h, _ptr(d_params), _ptr(d_X), _ptr(d_Y),
                                                   int(n), int(k), _ptr(d_pred), _ptr(d_grad),
                                                   _ptr(d_loss), _ptr(workspace), int(ws_bytes),
                                                   _stream(stream)))

    def get_mlp(self, dtype=F32):
        n = c_i32()
        self._check(self.L.kt_get_mlp(self.h, int(dtype), ctypes.byref(n), None))
        out = np.zeros(n.value, dtype=np.float32)
        self._check(self.L.kt_get_mlp(self.h, int(dtype), ctypes.byref(n), out.ctypes.data))
        return out

    # ------------------------------------------------------------ grouped
    @staticmethod
    def grouped_workspace_bytes(shapes) -> int:
        arr = shapes_array(shapes)
        b = c_sz()
        st = lib().kt_grouped_workspace_bytes(arr, len(shapes), ctypes.byref(b))
        if st != 0:
            raise KtError(st, "grouped workspace query")
        return b.value

    @staticmethod
    def _ptr_array(ptrs):
        arr = (c_vp * max(1, len(ptrs)))()
        for i, p in enumerate(ptrs):
            arr[i] = _ptr(p)
        return arr

    @staticmethod
    def _ld_array(ld, n):
        """Member leading dimensions: None (dense) or a list of (lda, ldb, ldc)."""
        if ld is None:
            return None
        a = np.ascontiguousarray(np.asarray(ld, dtype=np.int64).reshape(n, 3))
        return a

    @staticmethod
    def _opts_tuple(o):
        return (o.config_id, o.small_config_id, int(o.small_max_area), o.schedule, o.order,
                o.wgs_per_cu, o.pipeline)

    def grouped_plan(self, shapes, A, B, C, alpha=1.0, beta=0.0, opts=None, workspace=None,
                     ws_bytes=0, dtype=BF16, stream=None, ld=None):
        """shapes: list of (M, N, K); A, B, C: lists of device buffers; ld:
        None or per member (lda, ldb, ldc); opts: GroupedOpts or (config_id,
        small_config_id, small_max_area, schedule, order, wgs_per_cu[, pipeline[,
        visits]])."""
        arr = shapes_array([(m, n, k, 1, 0, 0) for (m, n, k) in shapes])
        plan = c_vp()
        o = None
        if opts is not None:
            o = opts if isinstance(opts, GroupedOpts) else GroupedOpts(*opts)
        lda = self._ld_array(ld, len(shapes))
        self._check(self.L.kt_grouped_plan_create(
            self.h, dtype, arr, len(shapes), self._ptr_array(A), self._ptr_array(B),
            self._ptr_array(C), None if lda is None else lda.ctypes.data, float(alpha), float(beta),
            None if o is None else ctypes.byref(o), _ptr(workspace), int(ws_bytes), _stream(stream),
            ctypes.byref(plan)))
        return plan

    def grouped_launch(self, plan, stream=None):
        self._check(self.L.kt_grouped_plan_launch(self.h, plan, _stream(stream)))

    def grouped_info(self, plan):
        n = c_i32()
        o = GroupedOpts()
        st = self.L.kt_grouped_plan_info(plan, ctypes.byref(n), ctypes.byref(o))
        if st != 0:
            raise KtError(st, "plan info")
        return n.value, self._opts_tuple(o)

    def grouped_destroy(self, plan):
        self.L.kt_grouped_plan_destroy(plan)

    def autotune_grouped(self, shapes, A, B, C, workspace, ws_bytes, dtype=BF16, stream=None,
                         ld=None):
        arr = shapes_array([(m, n, k, 1, 0, 0) for (m, n, k) in shapes])
        o = GroupedOpts()
        ms = c_f32()
        ev = c_i32()
        lda = self._ld_array(ld, len(shapes))
        self._check(self.L.kt_autotune_grouped(
            self.h, dtype, arr, len(shapes), self._ptr_array(A), self._ptr_array(B),
            self._ptr_array(C), None if lda is None else lda.ctypes.data, _ptr(workspace),
            int(ws_bytes), _stream(stream), ctypes.byref(o), ctypes.byref(ms), ctypes.byref(ev)))
        return self._opts_tuple(o), ms.value, ev.value
