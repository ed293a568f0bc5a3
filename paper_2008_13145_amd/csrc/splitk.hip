// Split-K GEMM: the K range of a deep product with few output tiles is cut
// into S slices, each slice is an ordinary GEMM into its own FP32 partial
// plane (alpha 1, beta 0, any compiled configuration), and one reduction
// pass adds the planes in slice order and applies alpha and beta.  This is
// the kernel type that section 3 names for tall-skinny products with a very
// deep K, where one tile per work-group leaves most compute units idle.
//
// Partial planes W[s][b][i][j] are dense (ld N, batch stride M*N, slice
// stride batch*M*N) in the caller's workspace.  With batch 1 the equal-depth
// slices run as one batched launch (slice index = batch index, A and B
// advanced by one slice depth per item); the ragged last slice, and every
// slice of a batched product, runs as a launch of its own.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>

#include "kt_internal.hpp"

namespace kt {

namespace {

constexpr int64_t SPLITK_ALIGN = 64;   // slice depth granule (a whole K tile of most configs)
constexpr int32_t SPLITK_MAX = 64;
constexpr int RED_THREADS = 256;

int64_t slice_depth(int64_t K, int32_t splits) {
  const int64_t kc = cdiv(K, splits);
  return cdiv(kc, SPLITK_ALIGN) * SPLITK_ALIGN;
}

size_t plane_bytes(const kt_shape* s) { return (size_t)s->batch * s->M * s->N * 4; }

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

// Automatic slice count: double S while the launch has fewer than
// AUTO_WG_TARGET work-groups (eight per compute unit: the products this is
// for are skinny and mostly wait on memory, so they want many loads in
// flight), the slices stay at least 256 deep and S < 64.  Hence
// S * tiles < 2 * AUTO_WG_TARGET, which bounds the workspace (below).
constexpr int64_t AUTO_WG_TARGET = 2048;

int32_t auto_splits(int64_t tiles, int64_t K) {
  int32_t S = 1;
  while (tiles * S < AUTO_WG_TARGET && S < SPLITK_MAX && K / (2 * S) >= 256) S *= 2;
  return S;
}

// Largest tile area of any configuration (256 x 256 low-precision tiles).
constexpr int64_t MAX_TILE_AREA = 256 * 256;

// C[b][i][j] = alpha * sum_s W[s][b][i][j] + beta * C[b][i][j]; C is not
// read when beta is 0.  An optional per-column bias (added after alpha and
// beta) and ReLU serve the convolution layers.  Each work-group covers
// RED_THREADS consecutive columns of one output row, so plane reads and C
// accesses are coalesced.
__global__ void __launch_bounds__(RED_THREADS)
splitk_reduce_kernel(const float* __restrict__ W, int32_t S, int64_t plane, int64_t M, int64_t N,
                     int64_t rows, float alpha, float beta, float* __restrict__ C, int64_t ldc,
                     int64_t sC, const float* __restrict__ bias, int32_t relu) {
  const int64_t col_blocks = (N + RED_THREADS - 1) / RED_THREADS;
  const int64_t total = rows * col_blocks;
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int64_t row = w / col_blocks;                 // b * M + i
    const int64_t j = (w - row * col_blocks) * RED_THREADS + threadIdx.x;
    if (j >= N) continue;
    const int64_t b = row / M, i = row - b * M;
    const float* p = W + row * N + j;
    float acc = 0.f;
    for (int32_t s = 0; s < S; ++s) acc += p[(int64_t)s * plane];
    float* c = C + b * sC + i * ldc + j;
    float out = alpha * acc;
    if (beta != 0.f) out = fmaf(beta, *c, out);
    if (bias) out += bias[j];
    *c = relu ? fmaxf(out, 0.f) : out;
  }
}

}  // namespace

}  // namespace kt

using namespace kt;

extern "C" {

kt_status kt_gemm_splitk_workspace_bytes(const kt_shape* s, int32_t splits, size_t* bytes) {
  if (!s || !bytes) return fail(nullptr, KT_EINVAL, "NULL argument");
  if (splits < 0 || splits > SPLITK_MAX) return fail(nullptr, KT_EINVAL, "need 0 <= splits <= 64");
  if (s->M < 0 || s->N < 0 || s->K < 0 || s->batch < 0)
    return fail(nullptr, KT_EINVAL, "negative M, N, K or batch");
  if (splits == 0) {   // automatic: S * plane <= S * tiles * tile area < 2 * target * MAX_TILE_AREA
    const size_t cap = (size_t)(2 * AUTO_WG_TARGET) * MAX_TILE_AREA * 4;
    const size_t all = (size_t)SPLITK_MAX * plane_bytes(s);
    *bytes = a256(all < cap ? all : cap);
    return KT_OK;
  }
  *bytes = splits == 1 ? 0 : a256((size_t)splits * plane_bytes(s));
  return KT_OK;
}

kt_status kt_gemm_splitk(kt_handle hh, kt_dtype dtype, const kt_shape* s, int32_t splits,
                         float alpha, const void* A, int64_t lda, int64_t strideA, const void* B,
                         int64_t ldb, int64_t strideB, float beta, float* C, int64_t ldc,
                         int64_t strideC, const float* scaleA, const float* scaleB,
                         int32_t config_id, void* workspace, size_t ws_bytes, void* stream,
                         int32_t* used_splits) {
  return kt::splitk_gemm(reinterpret_cast<Ctx*>(hh), dtype, s, splits, alpha, A, lda, strideA, B,
                         ldb, strideB, beta, C, ldc, strideC, scaleA, scaleB, config_id,
                         workspace, ws_bytes, stream, used_splits, nullptr, 0, nullptr);
}

}  // extern "C"

namespace kt {

// Slices a split-K variant really uses on shape s (slice depths are whole
// multiples of 64, so a shallow K takes fewer slices than asked for).
static int32_t effective_slices(const kt_shape* s, int32_t slices) {
  if (slices <= 1 || s->K <= 0) return 1;
  return (int32_t)cdiv(s->K, slice_depth(s->K, slices));
}

size_t split_plane_bytes(const kt_shape* s, int32_t slices) {
  const int32_t S = effective_slices(s, slices);
  if (S <= 1) return 0;
  const size_t need = a256((size_t)S * plane_bytes(s));
  return need <= SPLIT_PLANE_CAP ? need : 0;
}

size_t kernel_plane_bytes(const Ctx* h, int dtype, const kt_shape* s, int32_t id) {
  return split_plane_bytes(s, kernel_slices(h, dtype, id));
}

kt_status run_kernel(Ctx* h, int dtype, const kt_shape* s, float alpha, const void* A,
                     int64_t lda, int64_t sA, const void* B, int64_t ldb, int64_t sB, float beta,
                     float* C, int64_t ldc, int64_t sC, const float* scaleA, const float* scaleB,
                     int32_t id, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!valid_kernel(h, dtype, id))
    return fail(h, KT_EINVAL, "kernel id " + std::to_string(id) + " out of range");
  const int32_t base = kernel_base(h, dtype, id);
  const size_t need = kernel_plane_bytes(h, dtype, s, id);
  if (need == 0 || !ws || ws_bytes < need || s->M == 0 || s->N == 0 || s->batch == 0)
    return launch_gemm(h, dtype, s, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, scaleA,
                       scaleB, base, stream);
  return splitk_gemm(h, (kt_dtype)dtype, s, kernel_slices(h, dtype, id), alpha, A, lda, sA, B,
                     ldb, sB, beta, C, ldc, sC, scaleA, scaleB, base, ws, ws_bytes, stream,
                     nullptr, nullptr, 0, nullptr);
}

kt_status splitk_gemm(Ctx* h, kt_dtype dtype, const kt_shape* s, int32_t splits, float alpha,
                      const void* A, int64_t lda, int64_t strideA, const void* B, int64_t ldb,
                      int64_t strideB, float beta, float* C, int64_t ldc, int64_t strideC,
                      const float* scaleA, const float* scaleB, int32_t config_id,
                      void* workspace, size_t ws_bytes, void* stream, int32_t* used_splits,
                      const float* bias, int32_t relu, bool* epilogue_done) {
  if (epilogue_done) *epilogue_done = false;
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  if ((int)dtype < 0 || (int)dtype >= NUM_DTYPES) return fail(h, KT_EINVAL, "bad dtype");
  if (splits < 0 || splits > SPLITK_MAX) return fail(h, KT_EINVAL, "need 0 <= splits <= 64");
  kt_status st = check_gemm_args(h, s, lda, strideA, ldb, strideB, ldc, strideC);
  if (st != KT_OK) return st;
  if (used_splits) *used_splits = 1;
  if (s->M == 0 || s->N == 0 || s->batch == 0) return KT_OK;
  if (!C) return fail(h, KT_EINVAL, "C is NULL");
  if (s->K > 0 && (!A || !B)) return fail(h, KT_EINVAL, "A or B is NULL");
  if (dtype == KT_FP8E4M3 && (!scaleA || !scaleB))
    return fail(h, KT_EINVAL, "FP8 needs device scale pointers");
  if (config_id >= (int32_t)h->configs[dtype].size())
    return fail(h, KT_EINVAL, "config id out of range");
  hipStream_t stream_h = (hipStream_t)stream;

  const int64_t K = s->K;
  if (splits == 0) {   // automatic: the configuration first (selector on the whole product)
    if (config_id < 0) {
      if ((st = select_config(h, dtype, s, &config_id)) != KT_OK) return st;
      config_id = kernel_base(h, dtype, config_id);
    }
    const ConfigDef& c = h->configs[dtype][config_id];
    splits = auto_splits(cdiv(s->M, c.bm) * cdiv(s->N, c.bn) * s->batch, K);
  }
  const int64_t kc = K > 0 ? slice_depth(K, splits) : 0;
  const int32_t S = K > 0 ? (int32_t)cdiv(K, kc) : 1;
  if (S <= 1) {   // one slice: the plain product, no workspace
    int32_t cfg = config_id;
    if (cfg < 0) {
      if ((st = select_config(h, dtype, s, &cfg)) != KT_OK) return st;
      cfg = kernel_base(h, dtype, cfg);
    }
    return launch_gemm(h, dtype, s, alpha, A, lda, strideA, B, ldb, strideB, beta, C, ldc,
                       strideC, scaleA, scaleB, cfg, stream_h);
  }
  const int64_t plane = s->batch * s->M * s->N;
  if (!workspace || ws_bytes < (size_t)S * plane * 4)
    return fail(h, KT_EWORKSPACE, "split-K with " + std::to_string(S) + " slices needs " +
                                      std::to_string((size_t)S * plane * 4) +
                                      " bytes of partial planes (slices * batch * M * N floats), got " +
                                      std::to_string(workspace ? ws_bytes : 0));
  int32_t cfg = config_id;
  if (cfg < 0) {   // the selector sees the partial products as one batched GEMM
    kt_shape ps = *s;
    ps.K = kc;
    ps.batch = s->batch * S;
    if ((st = select_config(h, dtype, &ps, &cfg)) != KT_OK) return st;
    cfg = kernel_base(h, dtype, cfg);
  }
  const int eb = dtype == KT_F32 ? 4 : dtype == KT_BF16 ? 2 : 1;
  // element offsets of one slice depth along K in A and B
  const int64_t stepA = kc * (s->transA ? lda : 1);
  const int64_t stepB = kc * (s->transB ? 1 : ldb);
  const char* a0 = (const char*)A;
  const char* b0 = (const char*)B;
  float* W = (float*)workspace;
  const int64_t kl = K - (int64_t)(S - 1) * kc;   // depth of the last slice, 1..kc
  if (s->batch == 1) {
    const int32_t full = kl == kc ? S : S - 1;
    kt_shape ps = *s;
    ps.K = kc;
    ps.batch = full;
    st = launch_gemm(h, dtype, &ps, 1.f, a0, lda, stepA, b0, ldb, stepB, 0.f, W, s->N,
                     s->M * s->N, scaleA, scaleB, cfg, stream_h);
    if (st != KT_OK) return st;
    if (full < S) {
      ps.K = kl;
      ps.batch = 1;
      st = launch_gemm(h, dtype, &ps, 1.f, a0 + full * stepA * eb, lda, 0, b0 + full * stepB * eb,
                       ldb, 0, 0.f, W + (int64_t)full * plane, s->N, s->M * s->N, scaleA, scaleB,
                       cfg, stream_h);
      if (st != KT_OK) return st;
    }
  } else {
    for (int32_t q = 0; q < S; ++q) {
      kt_shape ps = *s;
      ps.K = q + 1 < S ? kc : kl;
      st = launch_gemm(h, dtype, &ps, 1.f, a0 + q * stepA * eb, lda, strideA,
                       b0 + q * stepB * eb, ldb, strideB, 0.f, W + (int64_t)q * plane, s->N,
                       s->M * s->N, scaleA, scaleB, cfg, stream_h);
      if (st != KT_OK) return st;
    }
  }
  const int64_t rows = s->batch * s->M;
  const int64_t blocks = rows * cdiv(s->N, RED_THREADS);
  const unsigned grid = (unsigned)(blocks < 65536 ? blocks : 65536);
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3(grid), dim3(RED_THREADS), 0, stream_h, W, S, plane,
                     s->M, s->N, rows, alpha, beta, C, ldc, strideC, bias, relu);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "split-K reduction launch");
  if (used_splits) *used_splits = S;
  if (epilogue_done) *epilogue_done = true;
  return KT_OK;
}

}  // namespace kt

// ---------------------------------------------------------------------------
// Split-K without allocation: the partial planes live in a static device
// array of NOALLOC_SCRATCH_BYTES that every GPU the library runs on holds
// until the process ends.  In host code `scratch` names a host-side stand-in,
// so its device address is looked up once per device (with that device
// current) and only that address is ever handed to kernels.
// ---------------------------------------------------------------------------

namespace kt {

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)32 << 20;
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) float scratch[NOALLOC_SCRATCH_BYTES / sizeof(float)];

std::mutex g_scratch_mu;
void* g_scratch_addr[MAX_DEVICES] = {};

}  // namespace

kt_status noalloc_scratch_init(Ctx* h) {
  if (h->device < 0) return KT_OK;
  if (h->device >= MAX_DEVICES) return fail(h, KT_EUNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[h->device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(h, e, "hipGetSymbolAddress(split-K scratch)");
    if (!p) return fail(h, KT_EHIP, "hipGetSymbolAddress returned NULL for the split-K scratch");
    g_scratch_addr[h->device] = p;
  }
  h->noalloc_scratch = g_scratch_addr[h->device];
  return KT_OK;
}

}  // namespace kt

extern "C" {

kt_status kt_gemm_splitk_noalloc_max_bytes(size_t* bytes) {
  if (!bytes) return fail(nullptr, KT_EINVAL, "NULL argument");
  *bytes = NOALLOC_SCRATCH_BYTES;
  return KT_OK;
}

kt_status kt_gemm_splitk_noalloc(kt_handle hh, kt_dtype dtype, const kt_shape* s, int32_t splits,
                                 float alpha, const void* A, int64_t lda, int64_t strideA,
                                 const void* B, int64_t ldb, int64_t strideB, float beta, float* C,
                                 int64_t ldc, int64_t strideC, const float* scaleA,
                                 const float* scaleB, int32_t config_id, void* stream,
                                 int32_t* used_splits) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  if (!h->noalloc_scratch) return fail(h, KT_EHIP, "split-K scratch address was not set up");
  h->forbid_alloc = true;
  kt_status st = splitk_gemm(h, dtype, s, splits, alpha, A, lda, strideA, B, ldb, strideB, beta,
                             C, ldc, strideC, scaleA, scaleB, config_id, h->noalloc_scratch,
                             NOALLOC_SCRATCH_BYTES, stream, used_splits, nullptr, 0, nullptr);
  h->forbid_alloc = false;
  if (st == KT_EWORKSPACE)
    h->err = "kt_gemm_splitk_noalloc: the static split-K scratch holds " +
             std::to_string(NOALLOC_SCRATCH_BYTES) + " bytes; " + h->err;
  return st;
}

}  // extern "C"
