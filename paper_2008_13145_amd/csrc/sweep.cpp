// Exhaustive configuration sweep (sections 3 and 3.1 of the paper): every
// kernel (configuration or split-K variant) is benchmarked on every problem
// -- a few warm-up launches, then a timed loop sized to a target duration,
// mean time per launch.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <numeric>
#include <thread>
#include <vector>

#include "kt_internal.hpp"

namespace kt {

static int64_t elem_bytes_of(int dtype) { return dtype == KT_F32 ? 4 : dtype == KT_BF16 ? 2 : 1; }

struct OperandPlan {
  int64_t lda, ldb, ldc, sA, sB, sC;
  size_t offA, offB, offC, offS, total;
};

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Operands of one problem, packed in a workspace: A, B (element type of the
// dtype), C (FP32), then for BF16 / FP8 an FP32 staging area the operands are
// generated in before conversion, and two FP8 scales plus the amax slot.
// Rows of A and B are dense, or with pad_rows rounded up to a multiple of 16
// elements (allocated in full), which puts every row on a 16-byte boundary
// in every dtype and keeps one layout for all of them.
static OperandPlan plan_for(const kt_shape& s, int dtype, bool pad_rows) {
  OperandPlan p;
  const int64_t eb = elem_bytes_of(dtype);
  const int64_t a_rows = s.transA ? s.K : s.M, a_cols = s.transA ? s.M : s.K;
  const int64_t b_rows = s.transB ? s.N : s.K, b_cols = s.transB ? s.K : s.N;
  auto ld_of = [&](int64_t cols) {
    const int64_t c = std::max<int64_t>(cols, 1);
    return pad_rows ? (c + 15) / 16 * 16 : c;
  };
  p.lda = ld_of(a_cols);
  p.ldb = ld_of(b_cols);
  p.ldc = std::max<int64_t>(s.N, 1);
  p.sA = a_rows * p.lda;
  p.sB = b_rows * p.ldb;
  p.sC = s.M * p.ldc;
  p.offA = 0;
  p.offB = align256(p.offA + (size_t)(s.batch * p.sA * eb));
  p.offC = align256(p.offB + (size_t)(s.batch * p.sB * eb));
  p.offS = align256(p.offC + (size_t)(s.batch * p.sC * 4));
  size_t stage = 0;
  if (dtype != KT_F32) stage = (size_t)std::max(s.batch * p.sA, s.batch * p.sB) * 4;
  p.total = align256(p.offS + 256 + stage);
  return p;
}

// Fill the operands of one problem (row r of a sweep) on the device.
static hipError_t fill_operands(int dtype, const OperandPlan& p, const kt_shape& s, char* ws,
                                uint64_t base, hipStream_t stream, Ctx* h) {
  float* C = (float*)(ws + p.offC);
  hipError_t e = fill_uniform(C, s.batch * p.sC, base + 2, 0, stream);
  if (e != hipSuccess) return e;
  if (dtype == KT_F32) {
    e = fill_uniform((float*)(ws + p.offA), s.batch * p.sA, base + 0, 0, stream);
    if (e == hipSuccess) e = fill_uniform((float*)(ws + p.offB), s.batch * p.sB, base + 1, 0, stream);
    return e;
  }
  float* stage = (float*)(ws + p.offS + 256);
  float* scales = (float*)(ws + p.offS);
  for (int which = 0; which < 2; ++which) {
    const int64_t n = s.batch * (which == 0 ? p.sA : p.sB);
    void* dst = ws + (which == 0 ? p.offA : p.offB);
    e = fill_uniform(stage, n, base + which, 0, stream);
    if (e != hipSuccess) return e;
    kt_status st;
    if (dtype == KT_BF16)
      st = kt_convert_bf16(reinterpret_cast<kt_handle>(h), stage, n, (uint16_t*)dst, stream);
    else
      st = kt_quantize_fp8(reinterpret_cast<kt_handle>(h), stage, n, (uint8_t*)dst, scales + which,
                           scales + 2, 16, stream);
    if (st != KT_OK) return hipErrorLaunchFailure;
  }
  return hipSuccess;
}

}  // namespace kt

using namespace kt;

extern "C" {

// Largest partial-plane need of any split-K variant of the dtype on shape s.
static size_t max_split_planes(int dtype, const kt_shape& s) {
  const DtypeRegistry& r = dtype_registry[dtype];
  size_t m = 0;
  for (int i = 0; i < r.n_splits; ++i) m = std::max(m, split_plane_bytes(&s, r.splits[i].slices));
  return m;
}

kt_status kt_sweep_workspace_bytes(const kt_shape* shapes, int32_t n_shapes, kt_dtype dtype,
                                   size_t* bytes) {
  if (!bytes || (n_shapes > 0 && !shapes) || n_shapes < 0) return KT_EINVAL;
  if ((int)dtype < 0 || (int)dtype > KT_FP8E4M3) return KT_EINVAL;
  size_t m = 0;
  for (int32_t i = 0; i < n_shapes; ++i) {
    if (shapes[i].M < 0 || shapes[i].N < 0 || shapes[i].K < 0 || shapes[i].batch < 0) return KT_EINVAL;
    // the padded layout bounds the dense one
    m = std::max(m, plan_for(shapes[i], dtype, true).total + max_split_planes(dtype, shapes[i]));
  }
  *bytes = m;
  return KT_OK;
}

kt_status kt_sweep(kt_handle hh, kt_dtype dtype, const kt_shape* shapes, int32_t n_shapes,
                   const int32_t* config_ids, int32_t n_configs, const kt_sweep_opts* opts,
                   void* workspace, size_t ws_bytes, void* stream_v, int64_t* time_ns) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  if ((int)dtype < 0 || (int)dtype > KT_FP8E4M3) return fail(h, KT_EINVAL, "bad dtype");
  if (n_shapes < 0 || (n_shapes > 0 && (!shapes || !time_ns)) || !opts)
    return fail(h, KT_EINVAL, "bad shapes / time_ns / opts");
  std::vector<int32_t> ids;
  if (config_ids) {
    if (n_configs < 0) return fail(h, KT_EINVAL, "n_configs < 0");
    ids.assign(config_ids, config_ids + n_configs);
  } else {
    ids.resize(num_kernels(h, dtype));
    std::iota(ids.begin(), ids.end(), 0);
    n_configs = (int32_t)ids.size();
  }
  for (int32_t id : ids)
    if (!valid_kernel(h, dtype, id)) return fail(h, KT_EINVAL, "kernel id out of range");
  if (opts->min_reps < 1 || opts->max_reps < opts->min_reps || opts->warmup < 0 ||
      opts->target_ms < 0 || (opts->pad_rows & ~1))
    return fail(h, KT_EINVAL, "bad sweep options");

  hipStream_t stream = (hipStream_t)stream_v;
  // Visit large work-group tiles first so the early cut has a tight
  // reference; split-K variants after every configuration.
  std::vector<int> order(ids.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const int32_t sa = kernel_slices(h, dtype, ids[a]), sb = kernel_slices(h, dtype, ids[b]);
    if ((sa > 1) != (sb > 1)) return sb > 1;
    const ConfigDef& ca = h->configs[dtype][kernel_base(h, dtype, ids[a])];
    const ConfigDef& cb = h->configs[dtype][kernel_base(h, dtype, ids[b])];
    const int64_t wa = (int64_t)ca.bm * ca.bn, wb = (int64_t)cb.bm * cb.bn;
    if (wa != wb) return wa > wb;
    return ca.t > cb.t;
  });
  hipEvent_t e0, e1;
  hipError_t he = hipEventCreate(&e0);
  if (he != hipSuccess) return hip_fail(h, he, "hipEventCreate");
  he = hipEventCreate(&e1);
  if (he != hipSuccess) { (void)hipEventDestroy(e0); return hip_fail(h, he, "hipEventCreate"); }
  kt_status result = KT_OK;
  // padded rows are allocated in full, which the DMA pipelines may rely on
  const bool keep_full_rows = h->full_rows;
  if (opts->pad_rows) h->full_rows = true;
  for (int32_t r = 0; r < n_shapes && result == KT_OK; ++r) {
    const kt_shape& s = shapes[r];
    int64_t* row = time_ns + (int64_t)r * n_configs;
    bool done = true;
    for (int32_t c = 0; c < n_configs; ++c) done = done && row[c] >= 0;
    if (done) continue;
    OperandPlan p = plan_for(s, dtype, opts->pad_rows != 0);
    size_t planes = 0;   // partial planes of the split-K kernels in the list
    for (int32_t id : ids) planes = std::max(planes, kernel_plane_bytes(h, dtype, &s, id));
    if (!workspace || ws_bytes < p.total + planes) {
      result = fail(h, KT_EWORKSPACE, "sweep workspace too small");
      break;
    }
    char* ws = (char*)workspace;
    const void* A = ws + p.offA;
    const void* B = ws + p.offB;
    float* C = (float*)(ws + p.offC);
    const float* scales = (const float*)(ws + p.offS);
    const uint64_t base = opts->seed * 0x100000001B3ull + (uint64_t)r * 4;
    he = fill_operands(dtype, p, s, ws, base, stream, h);
    if (he != hipSuccess) { result = fail(h, KT_EHIP, "operand fill / conversion failed"); break; }
    double best_ms = -1.0;
    for (int32_t c = 0; c < n_configs; ++c) if (row[c] > 0) {
      const double ms = row[c] * 1e-6;
      if (best_ms < 0 || ms < best_ms) best_ms = ms;
    }
    for (int oi = 0; oi < (int)order.size() && result == KT_OK; ++oi) {
      const int c = order[oi];
      if (row[c] >= 0) continue;
      const int32_t id = ids[c];
      auto launch = [&]() {
        return run_kernel(h, dtype, &s, opts->alpha, A, p.lda, p.sA, B, p.ldb, p.sB, opts->beta,
                          C, p.ldc, p.sC, scales, scales + 1, id, ws + p.total, planes, stream);
      };
      for (int w = 0; w < opts->warmup && result == KT_OK; ++w) result = launch();
      if (result != KT_OK) break;
      float ms_first = 0.f;
      if ((he = hipEventRecord(e0, stream)) != hipSuccess) { result = hip_fail(h, he, "event"); break; }
      if ((result = launch()) != KT_OK) break;
      if ((he = hipEventRecord(e1, stream)) != hipSuccess) { result = hip_fail(h, he, "event"); break; }
      if ((he = hipEventSynchronize(e1)) != hipSuccess) { result = hip_fail(h, he, "sync"); break; }
      (void)hipEventElapsedTime(&ms_first, e0, e1);
      double ms = ms_first;
      const bool cut = opts->cut_factor > 0 && best_ms > 0 && ms_first > opts->cut_factor * best_ms;
      if (!cut) {
        int reps = (int)ceil(opts->target_ms / std::max(ms_first, 1e-4f));
        reps = std::min(std::max(reps, opts->min_reps), opts->max_reps);
        if ((he = hipEventRecord(e0, stream)) != hipSuccess) { result = hip_fail(h, he, "event"); break; }
        for (int i = 0; i < reps && result == KT_OK; ++i) result = launch();
        if (result != KT_OK) break;
        if ((he = hipEventRecord(e1, stream)) != hipSuccess) { result = hip_fail(h, he, "event"); break; }
        if ((he = hipEventSynchronize(e1)) != hipSuccess) { result = hip_fail(h, he, "sync"); break; }
        float tot = 0.f;
        (void)hipEventElapsedTime(&tot, e0, e1);
        ms = tot / reps;
      }
      int64_t ns = (int64_t)llround(ms * 1e6);
      if (ns < 1) ns = 1;
      row[c] = ns;
      if (best_ms < 0 || ms < best_ms) best_ms = ms;
    }
    if (opts->pause_ms > 0)
      std::this_thread::sleep_for(std::chrono::microseconds((int64_t)(opts->pause_ms * 1000)));
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->full_rows = keep_full_rows;
  return result;
}

}  // extern "C"
