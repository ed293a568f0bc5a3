// C ABI entry points: handle, configuration tables, GEMM dispatch, operand fill.
#include <hip/hip_runtime.h>
#include <string.h>

#include <string>

#include "kt_internal.hpp"

namespace kt {

static thread_local std::string g_create_err;

kt_status fail(Ctx* h, kt_status st, const std::string& msg) {
  if (h) h->err = msg; else g_create_err = msg;
  return st;
}

kt_status hip_fail(Ctx* h, hipError_t e, const char* what) {
  return fail(h, KT_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool need_device(Ctx* h) {
  if (h->device < 0) {
    fail(h, KT_EINVAL, "this entry point launches GPU work; the handle was created without a device");
    return false;
  }
  return true;
}

int layout_index(int ta, int tb) { return (ta ? 2 : 0) + (tb ? 1 : 0); }

LaunchFn find_launcher(Ctx* h, int dtype, int32_t id, int ta, int tb) {
  if (dtype < 0 || dtype >= NUM_DTYPES) return nullptr;
  const auto& t = h->table[dtype];
  const int64_t at = (int64_t)id * 4 + layout_index(ta, tb);
  if (id < 0 || at >= (int64_t)t.size()) return nullptr;
  return t[at];
}

static void build_tables(Ctx* h) {
  for (int d = 0; d < NUM_DTYPES; ++d) {
    const DtypeRegistry& r = dtype_registry[d];
    h->configs[d].assign(r.configs, r.configs + r.n_configs);
    h->splits[d].assign(r.splits, r.splits + r.n_splits);
    h->table[d].assign((size_t)r.n_configs * 4, nullptr);
    for (int p = 0; p < r.n_parts; ++p) {
      const PartRef& pr = r.parts[p];
      if (!pr.entries) continue;
      for (int i = 0; i < *pr.count; ++i) {
        const LaunchEntry& e = pr.entries[i];
        h->table[d][(size_t)e.id * 4 + layout_index(e.ta, e.tb)] = e.fn;
      }
    }
  }
}

kt_status check_gemm_args(Ctx* h, const kt_shape* s, int64_t lda, int64_t sA, int64_t ldb,
                          int64_t sB, int64_t ldc, int64_t sC) {
  if (!s) return fail(h, KT_EINVAL, "shape is NULL");
  if (s->M < 0 || s->N < 0 || s->K < 0 || s->batch < 0)
    return fail(h, KT_EINVAL, "negative M, N, K or batch");
  if ((s->transA != 0 && s->transA != 1) || (s->transB != 0 && s->transB != 1))
    return fail(h, KT_EINVAL, "transA/transB must be 0 or 1");
  const int64_t M = s->M, N = s->N, K = s->K;
  const int64_t a_rows = s->transA ? K : M, a_cols = s->transA ? M : K;
  const int64_t b_rows = s->transB ? N : K, b_cols = s->transB ? K : N;
  auto max1 = [](int64_t v) { return v < 1 ? (int64_t)1 : v; };
  if (lda < max1(a_cols)) return fail(h, KT_EINVAL, "lda smaller than the stored row length of A");
  if (ldb < max1(b_cols)) return fail(h, KT_EINVAL, "ldb smaller than the stored row length of B");
  if (ldc < max1(N)) return fail(h, KT_EINVAL, "ldc < N");
  if (s->batch > 1) {
    if (sA != 0 && sA < a_rows * lda) return fail(h, KT_EINVAL, "strideA overlaps batch items (use 0 to broadcast)");
    if (sB != 0 && sB < b_rows * ldb) return fail(h, KT_EINVAL, "strideB overlaps batch items (use 0 to broadcast)");
    if (sC < M * ldc) return fail(h, KT_EINVAL, "strideC smaller than M * ldc");
  }
  if (sA < 0 || sB < 0 || sC < 0) return fail(h, KT_EINVAL, "negative batch stride");
  return KT_OK;
}

static int elem_bytes(int dtype) { return dtype == KT_F32 ? 4 : dtype == KT_BF16 ? 2 : 1; }

// Row alignment of an operand for the low-precision loaders: 2 = every row
// starts on a 4-byte boundary, 1 = only the base pointer does (rows are then
// loaded through a realigned window), 0 = neither (element loads); 3 = every
// row on a 16-byte boundary and whole 16-byte chunks along the contiguous
// extent `ext` (K for an operand stored K-contiguous, M or N otherwise),
// which takes the DMA pipeline.
int32_t operand_alignment(int dtype, const void* p, int64_t ld, int64_t stride, int64_t batch,
                          int64_t ext, bool full_rows) {
  const int eb = elem_bytes(dtype);
  if ((uintptr_t)p % 4 != 0) return 0;
  if ((ld * eb) % 4 != 0 || (stride * eb) % 4 != 0) return 1;
  const int64_t ce = 16 / eb;
  // with rows allocated in full, a row's last chunk may end anywhere within
  // the leading dimension
  const bool ext_ok = ext % ce == 0 || (full_rows && ext >= ce && ld >= (ext + ce - 1) / ce * ce);
  if ((uintptr_t)p % 16 == 0 && ld % ce == 0 && (batch <= 1 || stride % ce == 0) && ext_ok)
    return 3;
  return 2;
}

kt_status launch_gemm(Ctx* h, int dtype, const kt_shape* s, float alpha, const void* A,
                      int64_t lda, int64_t sA, const void* B, int64_t ldb, int64_t sB,
                      float beta, float* C, int64_t ldc, int64_t sC, const float* scaleA,
                      const float* scaleB, int32_t cfg, hipStream_t stream) {
  LaunchFn fn = find_launcher(h, dtype, cfg, s->transA, s->transB);
  if (!fn)
    return fail(h, KT_EUNSUPPORTED, "configuration " + std::to_string(cfg) + " for dtype " +
                                        std::to_string(dtype) + " and layout (" +
                                        std::to_string(s->transA) + "," +
                                        std::to_string(s->transB) + ") is not compiled");
  if (s->M == 0 || s->N == 0 || s->batch == 0) return KT_OK;
  const ConfigDef& c = h->configs[dtype][cfg];
  const int64_t tiles = cdiv(s->M, c.bm) * cdiv(s->N, c.bn);
  if (tiles > 0x7fffffffLL) return fail(h, KT_EINVAL, "problem too large for one grid");
  GemmArgs g;
  memset(&g, 0, sizeof g);
  g.M = s->M; g.N = s->N; g.K = s->K;
  g.lda = lda; g.sA = sA; g.ldb = ldb; g.sB = sB; g.ldc = ldc; g.sC = sC;
  g.alpha = alpha; g.beta = beta;
  g.scaleA = scaleA; g.scaleB = scaleB;
  g.vecA = operand_alignment(dtype, A, lda, sA, s->batch, s->transA ? s->M : s->K, h->full_rows);
  g.vecB = operand_alignment(dtype, B, ldb, sB, s->batch, s->transB ? s->K : s->N, h->full_rows);
  g.batch = s->batch;
  g.A = A;
  g.B = B;
  g.C = C;
  hipError_t e = fn(g, stream);   // splits huge batches into several grids
  if (e != hipSuccess) return hip_fail(h, e, "kernel launch");
  return KT_OK;
}

}  // namespace kt

using namespace kt;

extern "C" {

int32_t kt_abi_version(void) { return 111; }

kt_status kt_create(kt_handle* out, int device) {
  if (!out) return fail(nullptr, KT_EINVAL, "out is NULL");
  *out = nullptr;
  Ctx* h = new (std::nothrow) Ctx();
  if (!h) return fail(nullptr, KT_EINVAL, "out of host memory");
  if (device >= 0) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) {
      delete h;
      return fail(nullptr, KT_EHIP, std::string("no HIP device: ") + hipGetErrorString(e));
    }
    if (device >= n) {
      delete h;
      return fail(nullptr, KT_EINVAL, "device index out of range");
    }
    e = hipSetDevice(device);
    if (e != hipSuccess) {
      delete h;
      return fail(nullptr, KT_EHIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    }
    hipDeviceProp_t p;
    e = hipGetDeviceProperties(&p, device);
    if (e != hipSuccess) {
      delete h;
      return fail(nullptr, KT_EHIP, std::string("hipGetDeviceProperties: ") + hipGetErrorString(e));
    }
    if (strncmp(p.gcnArchName, "gfx950", 6) != 0) {
      delete h;
      return fail(nullptr, KT_EUNSUPPORTED, std::string("kernels are built for gfx950, device is ") + p.gcnArchName);
    }
  } else if (device != -1) {
    delete h;
    return fail(nullptr, KT_EINVAL, "device must be >= 0 or -1 (host only)");
  }
  h->device = device;
  build_tables(h);
  if (device >= 0) {
    kt_status st = noalloc_scratch_init(h);
    if (st != KT_OK) {
      g_create_err = h->err;
      delete h;
      return st;
    }
  }
  *out = reinterpret_cast<kt_handle>(h);
  return KT_OK;
}

kt_status kt_destroy(kt_handle hh) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return KT_OK;
  if (h->device >= 0) {
    (void)hipSetDevice(h->device);
    for (int d = 0; d < NUM_DTYPES; ++d) free_selector_device(h, d);
    if (h->scratch) (void)hipFree(h->scratch);
    if (h->d_lut) (void)hipFree(h->d_lut);
  }
  delete h;
  return KT_OK;
}

const char* kt_last_error(kt_handle hh) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  return h ? h->err.c_str() : g_create_err.c_str();
}

kt_status kt_num_configs(kt_handle hh, kt_dtype dtype, int32_t* n) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h || !n) return fail(h, KT_EINVAL, "NULL argument");
  if ((int)dtype < 0 || (int)dtype >= NUM_DTYPES) return fail(h, KT_EINVAL, "bad dtype");
  *n = (int32_t)h->configs[dtype].size();
  return KT_OK;
}

kt_status kt_get_config(kt_handle hh, kt_dtype dtype, int32_t id, kt_config* out) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h || !out) return fail(h, KT_EINVAL, "NULL argument");
  if ((int)dtype < 0 || (int)dtype >= NUM_DTYPES) return fail(h, KT_EINVAL, "bad dtype");
  if (id < 0 || id >= (int32_t)h->configs[dtype].size()) return fail(h, KT_EINVAL, "config id out of range");
  const ConfigDef& c = h->configs[dtype][id];
  out->bm = c.bm; out->bn = c.bn; out->t = c.t; out->bk = c.bk; out->dtype = dtype;
  return KT_OK;
}

kt_status kt_config_compiled(kt_handle hh, kt_dtype dtype, int32_t id, int32_t ta, int32_t tb,
                             int32_t* compiled) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h || !compiled) return fail(h, KT_EINVAL, "NULL argument");
  *compiled = valid_kernel(h, dtype, id) &&
              find_launcher(h, dtype, kernel_base(h, dtype, id), ta, tb) != nullptr;
  return KT_OK;
}

kt_status kt_num_kernels(kt_handle hh, kt_dtype dtype, int32_t* n) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h || !n) return fail(h, KT_EINVAL, "NULL argument");
  if ((int)dtype < 0 || (int)dtype >= NUM_DTYPES) return fail(h, KT_EINVAL, "bad dtype");
  *n = num_kernels(h, dtype);
  return KT_OK;
}

kt_status kt_get_kernel(kt_handle hh, kt_dtype dtype, int32_t id, kt_config* cfg, int32_t* base_id,
                        int32_t* slices) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h || !cfg || !base_id || !slices) return fail(h, KT_EINVAL, "NULL argument");
  if ((int)dtype < 0 || (int)dtype >= NUM_DTYPES) return fail(h, KT_EINVAL, "bad dtype");
  if (!valid_kernel(h, dtype, id)) return fail(h, KT_EINVAL, "kernel id out of range");
  *base_id = kernel_base(h, dtype, id);
  *slices = kernel_slices(h, dtype, id);
  const ConfigDef& c = h->configs[dtype][*base_id];
  cfg->bm = c.bm; cfg->bn = c.bn; cfg->t = c.t; cfg->bk = c.bk; cfg->dtype = dtype;
  return KT_OK;
}

kt_status kt_set_workspace(kt_handle hh, void* workspace, size_t bytes) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!workspace && bytes) return fail(h, KT_EINVAL, "NULL workspace with a nonzero size");
  h->gemm_ws = workspace;
  h->gemm_ws_bytes = workspace ? bytes : 0;
  return KT_OK;
}

kt_status kt_kernel_workspace_bytes(kt_handle hh, kt_dtype dtype, const kt_shape* s, int32_t id,
                                    size_t* bytes) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h || !s || !bytes) return fail(h, KT_EINVAL, "NULL argument");
  if ((int)dtype < 0 || (int)dtype >= NUM_DTYPES) return fail(h, KT_EINVAL, "bad dtype");
  if (!valid_kernel(h, dtype, id)) return fail(h, KT_EINVAL, "kernel id out of range");
  if (s->M < 0 || s->N < 0 || s->K < 0 || s->batch < 0)
    return fail(h, KT_EINVAL, "negative M, N, K or batch");
  *bytes = kernel_plane_bytes(h, dtype, s, id);
  return KT_OK;
}

kt_status kt_gemm(kt_handle hh, kt_dtype in_dtype, const kt_shape* s, float alpha, const void* A,
                  int64_t lda, int64_t strideA, const void* B, int64_t ldb, int64_t strideB,
                  float beta, float* C, int64_t ldc, int64_t strideC, const float* scaleA,
                  const float* scaleB, int32_t config_id, void* stream) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  if ((int)in_dtype < 0 || (int)in_dtype >= NUM_DTYPES) return fail(h, KT_EINVAL, "bad dtype");
  kt_status st = check_gemm_args(h, s, lda, strideA, ldb, strideB, ldc, strideC);
  if (st != KT_OK) return st;
  if (s->M == 0 || s->N == 0 || s->batch == 0) return KT_OK;
  if (!C) return fail(h, KT_EINVAL, "C is NULL");
  if (s->K > 0 && (!A || !B)) return fail(h, KT_EINVAL, "A or B is NULL");
  if (in_dtype == KT_FP8E4M3 && (!scaleA || !scaleB))
    return fail(h, KT_EINVAL, "FP8 needs device scale pointers");
  int32_t id = config_id;
  if (id < 0) {
    st = select_config(h, in_dtype, s, &id);
    if (st != KT_OK) return st;
  }
  if (!valid_kernel(h, in_dtype, id)) return fail(h, KT_EINVAL, "kernel id out of range");
  return run_kernel(h, in_dtype, s, alpha, A, lda, strideA, B, ldb, strideB, beta, C, ldc,
                    strideC, scaleA, scaleB, id, h->gemm_ws, h->gemm_ws_bytes, (hipStream_t)stream);
}

kt_status kt_dma_pipeline(kt_handle hh, kt_dtype dtype, const kt_shape* s, const void* A,
                         int64_t lda, int64_t strideA, const void* B, int64_t ldb, int64_t strideB,
                         int32_t* dma) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!s || !dma) return fail(h, KT_EINVAL, "NULL argument");
  if ((int)dtype < 0 || (int)dtype >= NUM_DTYPES) return fail(h, KT_EINVAL, "bad dtype");
  *dma = operand_alignment(dtype, A, lda, strideA, s->batch, s->transA ? s->M : s->K,
                           h->full_rows) == 3 &&
         operand_alignment(dtype, B, ldb, strideB, s->batch, s->transB ? s->K : s->N,
                           h->full_rows) == 3;
  return KT_OK;
}

kt_status kt_set_full_rows(kt_handle hh, int32_t enabled) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (enabled != 0 && enabled != 1) return fail(h, KT_EINVAL, "enabled must be 0 or 1");
  h->full_rows = enabled != 0;
  return KT_OK;
}

kt_status kt_fill_uniform(kt_handle hh, float* dst, int64_t n, uint64_t seed, int64_t offset,
                          void* stream) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  if (n < 0 || offset < 0) return fail(h, KT_EINVAL, "negative size or offset");
  if (n == 0) return KT_OK;
  if (!dst) return fail(h, KT_EINVAL, "dst is NULL");
  hipError_t e = fill_uniform(dst, n, seed, offset, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(h, e, "fill launch");
  return KT_OK;
}

}  // extern "C"
