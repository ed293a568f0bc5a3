// Internal state of a kt handle and helpers shared by the host sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/kt.h"
#include "gemm_f32.hpp"
#include "registry.hpp"

namespace kt {

enum { NUM_DTYPES = 3 };

struct Tree {
  std::vector<int32_t> feature, left, right, cls;
  std::vector<int64_t> threshold;
};

struct MlpModel {
  int32_t k = 0;
  std::vector<float> params;   // W1 b1 W2 b2 W3 b3 packed
};

struct ShapeKey {
  int64_t M, N, K, batch;
  int32_t ta, tb, dtype;
  bool operator<(const ShapeKey& o) const {
    return std::tie(M, N, K, batch, ta, tb, dtype) < std::tie(o.M, o.N, o.K, o.batch, o.ta, o.tb, o.dtype);
  }
};

// Selector state of one dtype (each dtype has its own configuration space,
// sweep table, pruned set and selector).
struct SelState {
  int32_t kind = -1;               // kt_selector, -1 = none
  std::vector<int32_t> chosen;     // deployed configuration ids
  Tree tree;
  MlpModel mlp;
  void* d_tree = nullptr;          // device copy of the tree for batch selection
  size_t d_tree_bytes = 0;
  void* d_mlp = nullptr;           // device copy of the MLP weights + chosen ids
  std::map<ShapeKey, int32_t> exhaustive_cache;
  // Training box of a fitted model: the smallest and largest M, N, K and
  // batch it was fitted on.  Shapes outside it are timed over the chosen
  // configurations instead of trusting the model (when fallback is on).
  bool have_box = false;
  int64_t box_lo[4] = {0, 0, 0, 0}, box_hi[4] = {0, 0, 0, 0};
  int32_t fallback = 1;
  std::map<ShapeKey, int32_t> fallback_cache;
};

struct Ctx {
  int device = -1;
  std::string err;
  // launcher lookup: [dtype][id * 4 + layout]
  std::vector<LaunchFn> table[NUM_DTYPES];
  std::vector<ConfigDef> configs[NUM_DTYPES];
  std::vector<SplitDef> splits[NUM_DTYPES];   // split-K variants after the configurations
  SelState sel[NUM_DTYPES];
  void* scratch = nullptr;         // exhaustive-selection operands (handle-owned)
  size_t scratch_bytes = 0;
  std::vector<uint16_t> sigmoid_lut;
  void* d_lut = nullptr;           // device sigmoid table (handle-owned)
  kt_grouped_opts grouped_best{};  // autotuner result for grouped GEMM
  bool grouped_tuned = false;
  void* gemm_ws = nullptr;         // caller's workspace for split-K kernels run by kt_gemm
  size_t gemm_ws_bytes = 0;
  void* noalloc_scratch = nullptr; // device address of the static split-K scratch
  bool forbid_alloc = false;       // set while an entry point that must not allocate runs
  bool full_rows = false;          // caller: every operand row is allocated to its full ld
};

// Record an error message on the handle and return the status.
kt_status fail(Ctx* h, kt_status st, const std::string& msg);
kt_status hip_fail(Ctx* h, hipError_t e, const char* what);
bool need_device(Ctx* h);
LaunchFn find_launcher(Ctx* h, int dtype, int32_t id, int ta, int tb);
int layout_index(int ta, int tb);

// Shape validation shared by gemm and sweep; returns KT_OK or KT_EINVAL with a message.
kt_status check_gemm_args(Ctx* h, const kt_shape* s, int64_t lda, int64_t sA, int64_t ldb,
                          int64_t sB, int64_t ldc, int64_t sC);
// Launch one GEMM with a given configuration (no validation beyond lookup).
kt_status launch_gemm(Ctx* h, int dtype, const kt_shape* s, float alpha, const void* A,
                      int64_t lda, int64_t sA, const void* B, int64_t ldb, int64_t sB,
                      float beta, float* C, int64_t ldc, int64_t sC, const float* scaleA,
                      const float* scaleB, int32_t cfg, hipStream_t stream);

// Alignment class of an operand (GemmArgs::vecA / vecB).
int32_t operand_alignment(int dtype, const void* p, int64_t ld, int64_t stride, int64_t batch,
                          int64_t ext, bool full_rows);

// Kernel ids: configurations 0 .. n_configs-1, then split-K variants.
inline int32_t num_kernels(const Ctx* h, int dtype) {
  return (int32_t)(h->configs[dtype].size() + h->splits[dtype].size());
}
inline bool valid_kernel(const Ctx* h, int dtype, int32_t id) {
  return dtype >= 0 && dtype < NUM_DTYPES && id >= 0 && id < num_kernels(h, dtype);
}
// The configuration a kernel runs (the kernel itself, or a variant's base).
inline int32_t kernel_base(const Ctx* h, int dtype, int32_t id) {
  const int32_t nc = (int32_t)h->configs[dtype].size();
  return id < nc ? id : h->splits[dtype][id - nc].base;
}
inline int32_t kernel_slices(const Ctx* h, int dtype, int32_t id) {
  const int32_t nc = (int32_t)h->configs[dtype].size();
  return id < nc ? 1 : h->splits[dtype][id - nc].slices;
}

// Partial planes of a split-K kernel never exceed this (beyond it, or beyond
// the workspace at hand, the variant runs as its base configuration unsplit).
constexpr size_t SPLIT_PLANE_CAP = (size_t)256 << 20;

// Bytes of partial planes kernel `id` uses on shape s (0 when it runs unsplit
// with an unlimited workspace).
size_t kernel_plane_bytes(const Ctx* h, int dtype, const kt_shape* s, int32_t id);
// The same for a slice count (no handle needed).
size_t split_plane_bytes(const kt_shape* s, int32_t slices);

// Run kernel `id` (a configuration or a split-K variant; the variant gets
// the workspace [ws, ws + ws_bytes) for its partial planes and runs unsplit
// when they do not fit).  No validation beyond lookup.
kt_status run_kernel(Ctx* h, int dtype, const kt_shape* s, float alpha, const void* A,
                     int64_t lda, int64_t sA, const void* B, int64_t ldb, int64_t sB, float beta,
                     float* C, int64_t ldc, int64_t sC, const float* scaleA, const float* scaleB,
                     int32_t id, void* ws, size_t ws_bytes, hipStream_t stream);

// Fill kernel launcher (device).
hipError_t fill_uniform(float* dst, int64_t n, uint64_t seed, int64_t offset, hipStream_t s);

// Selector helpers (select.hip, mlp.hip); dtype picks the selector state.
kt_status select_config(Ctx* h, int dtype, const kt_shape* s, int32_t* id);
kt_status mlp_select_host(Ctx* h, int dtype, const kt_shape* s, int32_t* id);
kt_status mlp_select_batch(Ctx* h, int dtype, const kt_shape* d_shapes, int32_t n, int32_t* d_ids,
                           hipStream_t st);
kt_status mlp_upload(Ctx* h, int dtype);
kt_status fit_mlp(Ctx* h, int dtype, const kt_shape* shapes, const int64_t* time_ns, int32_t n,
                  int32_t d, const int32_t* chosen, int32_t k, const kt_mlp_opts* o, void* ws,
                  size_t ws_bytes, hipStream_t st);
void free_selector_device(Ctx* h, int dtype);

// Normalize a host time table on the GPU (workspace of
// kt_prune_workspace_bytes(n, d, 1, 1) or more) and copy the Q16 result to
// host memory; synchronizes the stream.
kt_status normalize_table_host(Ctx* h, const int64_t* time_ns, int32_t n, int32_t d, kt_norm norm,
                               void* workspace, size_t ws_bytes, hipStream_t st, uint16_t* out);

// Looks up the device address of the static split-K scratch for the handle's
// device (once per device, that device current) and keeps it on the handle.
kt_status noalloc_scratch_init(Ctx* h);

// Sigmoid lookup table of the normalization (Q16 -> Q16).
const std::vector<uint16_t>& sigmoid_table(Ctx* h);

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// kt_gemm_splitk with an optional per-column bias and ReLU applied by the
// reduction pass; *epilogue_done reports whether that pass ran (with a single
// slice the plain GEMM runs and the caller applies bias and activation).
kt_status splitk_gemm(Ctx* h, kt_dtype dtype, const kt_shape* s, int32_t splits, float alpha,
                      const void* A, int64_t lda, int64_t strideA, const void* B, int64_t ldb,
                      int64_t strideB, float beta, float* C, int64_t ldc, int64_t strideC,
                      const float* scaleA, const float* scaleB, int32_t config_id,
                      void* workspace, size_t ws_bytes, void* stream, int32_t* used_splits,
                      const float* bias, int32_t relu, bool* epilogue_done);

}  // namespace kt
