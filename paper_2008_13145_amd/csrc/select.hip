// Runtime kernel selection (section 5 of the paper, "Deploying the kernels").
//
// Each training problem is labelled with the chosen kernel that ran it
// fastest, and a decision tree on the matrix sizes learns that label
// (section 5.1, trees A/B/C).  At launch time the tree is walked -- the
// paper's nested if statements in the kernel launcher -- to pick one of the
// deployed configurations.  Exhaustive search (time every compiled
// configuration once per unseen shape, then cache) is the fallback selector
// and the reference that a selector's regret is measured against.
//
// Integer CART: features (M, N, K, batch, transA, transB) as raw integers;
// Gini criterion with splits scored by S = A/n_L + B/n_R (A, B the sums of
// squared class counts of each side), compared exactly by cross-
// multiplication; thresholds floor(sqrt(a*b)) between consecutive distinct
// values; x <= t goes left; first maximum over features 0..5 and ascending
// thresholds; a split must strictly beat the parent's sum(n_c^2)/n; leaves
// predict the majority class (lowest on ties); nodes in pre-order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <fstream>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "kt_internal.hpp"

namespace kt {

typedef __int128 i128;

static uint64_t isqrt_u64(uint64_t p) {
  uint64_t r = (uint64_t)sqrtl((long double)p);
  while ((i128)r * r > (i128)p) --r;
  while ((i128)(r + 1) * (r + 1) <= (i128)p) ++r;
  return r;
}

struct CartData {
  std::vector<std::array<int64_t, 6>> X;
  std::vector<int32_t> y;
  int n_classes;
  int max_depth;    // < 0: unlimited
  int min_leaf;
};

static int32_t cart_build(const CartData& D, std::vector<int32_t>& idx, int depth, Tree& T) {
  const int32_t node = (int32_t)T.feature.size();
  T.feature.push_back(-1);
  T.threshold.push_back(0);
  T.left.push_back(-1);
  T.right.push_back(-1);
  T.cls.push_back(0);
  const int nc = D.n_classes;
  std::vector<int64_t> cnt(nc, 0);
  for (int32_t i : idx) cnt[D.y[i]]++;
  int best_c = 0;
  for (int c = 1; c < nc; ++c) if (cnt[c] > cnt[best_c]) best_c = c;
  T.cls[node] = best_c;
  const int64_t n = (int64_t)idx.size();
  int nonzero = 0;
  for (int c = 0; c < nc; ++c) nonzero += cnt[c] > 0;
  if (nonzero <= 1 || (D.max_depth >= 0 && depth >= D.max_depth) || n < 2 * (int64_t)D.min_leaf)
    return node;
  bool have = false;
  i128 bnum = 0, bden = 1;
  int bf = -1;
  int64_t bt = 0;
  std::vector<int32_t> order(idx);
  std::vector<int64_t> cl(nc), cr(nc);
  for (int f = 0; f < 6; ++f) {
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return D.X[a][f] < D.X[b][f]; });
    std::fill(cl.begin(), cl.end(), 0);
    cr = cnt;
    int64_t pos = 0;
    while (pos < n) {
      const int64_t v = D.X[order[pos]][f];
      while (pos < n && D.X[order[pos]][f] == v) {
        cl[D.y[order[pos]]]++;
        cr[D.y[order[pos]]]--;
        ++pos;
      }
      if (pos == n) break;
      const int64_t a = v, b = D.X[order[pos]][f];
      const int64_t t = (int64_t)isqrt_u64((uint64_t)a * (uint64_t)b);
      const int64_t nl = pos, nr = n - pos;
      if (nl < D.min_leaf || nr < D.min_leaf) continue;
      i128 A = 0, B = 0;
      for (int c = 0; c < nc; ++c) { A += (i128)cl[c] * cl[c]; B += (i128)cr[c] * cr[c]; }
      const i128 num = A * nr + B * nl, den = (i128)nl * nr;
      if (!have || num * bden > bnum * den) {
        have = true; bnum = num; bden = den; bf = f; bt = t;
      }
    }
  }
  if (!have) return node;
  i128 P = 0;
  for (int c = 0; c < nc; ++c) P += (i128)cnt[c] * cnt[c];
  if (!(bnum * n > P * bden)) return node;
  T.feature[node] = bf;
  T.threshold[node] = bt;
  std::vector<int32_t> li, ri;
  for (int32_t i : idx) (D.X[i][bf] <= bt ? li : ri).push_back(i);
  idx.clear();
  idx.shrink_to_fit();
  const int32_t l = cart_build(D, li, depth + 1, T);
  T.left[node] = l;
  const int32_t r = cart_build(D, ri, depth + 1, T);
  T.right[node] = r;
  return node;
}

static inline int64_t feat(const kt_shape& s, int f) {
  switch (f) {
    case 0: return s.M;
    case 1: return s.N;
    case 2: return s.K;
    case 3: return s.batch;
    case 4: return s.transA;
    default: return s.transB;
  }
}

static int32_t tree_walk(const Tree& T, const kt_shape& s) {
  int32_t node = 0;
  while (T.feature[node] >= 0)
    node = feat(s, T.feature[node]) <= T.threshold[node] ? T.left[node] : T.right[node];
  return T.cls[node];
}

// Device tree walk for a batch of shapes.  Layout of the packed buffer:
// int64 threshold[n], int32 feature[n], left[n], right[n], cls[n], chosen[k].
__global__ void select_tree_kernel(const kt_shape* __restrict__ shapes, int32_t n,
                                   const char* __restrict__ tree, int32_t n_nodes, int32_t k,
                                   int32_t* __restrict__ ids) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t* thr = (const int64_t*)tree;
  const int32_t* fea = (const int32_t*)(thr + n_nodes);
  const int32_t* lef = fea + n_nodes;
  const int32_t* rig = lef + n_nodes;
  const int32_t* cls = rig + n_nodes;
  const int32_t* chosen = cls + n_nodes;
  const kt_shape s = shapes[i];
  int32_t node = 0;
  for (int32_t step = 0; step < n_nodes && fea[node] >= 0; ++step) {
    const int f = fea[node];
    const int64_t x = f == 0 ? s.M : f == 1 ? s.N : f == 2 ? s.K : f == 3 ? s.batch
                    : f == 4 ? (int64_t)s.transA : (int64_t)s.transB;
    node = x <= thr[node] ? lef[node] : rig[node];
  }
  const int32_t c = cls[node];
  ids[i] = (c >= 0 && c < k) ? chosen[c] : -1;
}

void free_selector_device(Ctx* h, int dtype) {
  SelState& S = h->sel[dtype];
  if (h->device >= 0) {
    if (S.d_tree) (void)hipFree(S.d_tree);
    if (S.d_mlp) (void)hipFree(S.d_mlp);
  }
  S.d_tree = nullptr;
  S.d_tree_bytes = 0;
  S.d_mlp = nullptr;
}

static kt_status upload_tree(Ctx* h, int dtype) {
  SelState& S = h->sel[dtype];
  if (h->device < 0) return KT_OK;
  free_selector_device(h, dtype);
  const size_t nn = S.tree.feature.size();
  const size_t bytes = nn * 8 + nn * 4 * 4 + S.chosen.size() * 4;
  std::vector<char> buf(bytes);
  char* p = buf.data();
  memcpy(p, S.tree.threshold.data(), nn * 8); p += nn * 8;
  memcpy(p, S.tree.feature.data(), nn * 4); p += nn * 4;
  memcpy(p, S.tree.left.data(), nn * 4); p += nn * 4;
  memcpy(p, S.tree.right.data(), nn * 4); p += nn * 4;
  memcpy(p, S.tree.cls.data(), nn * 4); p += nn * 4;
  memcpy(p, S.chosen.data(), S.chosen.size() * 4);
  hipError_t e = hipMalloc(&S.d_tree, bytes);
  if (e != hipSuccess) { S.d_tree = nullptr; return hip_fail(h, e, "hipMalloc tree"); }
  e = hipMemcpy(S.d_tree, buf.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(h, e, "upload tree");
  S.d_tree_bytes = bytes;
  return KT_OK;
}

static int64_t elem_bytes_sel(int dtype) { return dtype == KT_F32 ? 4 : dtype == KT_BF16 ? 2 : 1; }

// Time the candidate kernels (those whose configuration is compiled for the
// shape's layout) on handle-owned scratch operands (generated in FP32 and
// converted for BF16 / FP8), split-K variants with scratch partial planes:
// one untimed launch, then three timed ones each; the fastest (first on
// ties) wins.  Allocates the scratch on first use and synchronizes.
static kt_status time_candidates(Ctx* h, int dtype, const kt_shape* s,
                                 const std::vector<int32_t>& cands, int32_t* out) {
  if (!need_device(h)) return KT_EINVAL;
  if (h->forbid_alloc)
    return fail(h, KT_EUNSUPPORTED, "the exhaustive selector would allocate scratch operands for "
                                    "an unseen shape; this entry point allocates nothing (select "
                                    "the shape once with kt_select first, or pass a config id)");
  const int64_t eb = elem_bytes_sel(dtype);
  const int64_t a_rows = s->transA ? s->K : s->M, a_cols = s->transA ? s->M : s->K;
  const int64_t b_rows = s->transB ? s->N : s->K, b_cols = s->transB ? s->K : s->N;
  // rows padded to 16 elements when the caller promises whole rows (the
  // sweep's padded layout), else dense
  auto ld_of = [&](int64_t cols) {
    const int64_t c = std::max<int64_t>(cols, 1);
    return h->full_rows ? (c + 15) / 16 * 16 : c;
  };
  const int64_t lda = ld_of(a_cols), ldb = ld_of(b_cols);
  const int64_t ldc = std::max<int64_t>(s->N, 1);
  const int64_t nA = s->batch * a_rows * lda, nB = s->batch * b_rows * ldb, nC = s->batch * s->M * ldc;
  auto r256 = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
  const int64_t offB = r256(nA * eb), offC = offB + r256(nB * eb), offS = offC + r256(nC * 4);
  const int64_t offT = offS + 256;   // FP32 staging for BF16 / FP8 operands
  const int64_t offW = offT + r256(dtype == KT_F32 ? 0 : std::max(nA, nB) * 4);   // split-K planes
  size_t planes = 0;
  for (int32_t id : cands) planes = std::max(planes, kernel_plane_bytes(h, dtype, s, id));
  const size_t need = (size_t)offW + planes + 256;
  if (h->scratch_bytes < need) {
    if (h->scratch) (void)hipFree(h->scratch);
    h->scratch = nullptr;
    h->scratch_bytes = 0;
    hipError_t e = hipMalloc(&h->scratch, need);
    if (e != hipSuccess) return hip_fail(h, e, "hipMalloc exhaustive-selection scratch");
    h->scratch_bytes = need;
  }
  char* base = (char*)h->scratch;
  void* A = base;
  void* B = base + offB;
  float* C = (float*)(base + offC);
  float* scales = (float*)(base + offS);
  hipError_t e = hipSuccess;
  if (dtype == KT_F32) {
    e = fill_uniform((float*)A, nA, 1, 0, nullptr);
    if (e == hipSuccess) e = fill_uniform((float*)B, nB, 2, 0, nullptr);
    if (e != hipSuccess) return hip_fail(h, e, "fill");
  } else {
    float* stage = (float*)(base + offT);
    for (int which = 0; which < 2; ++which) {
      const int64_t n = which == 0 ? nA : nB;
      void* dst = which == 0 ? A : B;
      e = fill_uniform(stage, n, 1 + which, 0, nullptr);
      if (e != hipSuccess) return hip_fail(h, e, "fill");
      kt_status st = dtype == KT_BF16
          ? kt_convert_bf16(reinterpret_cast<kt_handle>(h), stage, n, (uint16_t*)dst, nullptr)
          : kt_quantize_fp8(reinterpret_cast<kt_handle>(h), stage, n, (uint8_t*)dst, scales + which,
                            scales + 2, 16, nullptr);
      if (st != KT_OK) return st;
    }
  }
  hipEvent_t e0, e1;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(h, e, "event");
  if ((e = hipEventCreate(&e1)) != hipSuccess) { (void)hipEventDestroy(e0); return hip_fail(h, e, "event"); }
  int32_t best = -1;
  float best_ms = 0.f;
  kt_status st = KT_OK;
  for (size_t ci = 0; ci < cands.size() && st == KT_OK; ++ci) {
    const int32_t id = cands[ci];
    if (!find_launcher(h, dtype, kernel_base(h, dtype, id), s->transA, s->transB)) continue;
    auto launch = [&]() {
      return run_kernel(h, dtype, s, 1.f, A, lda, a_rows * lda, B, ldb, b_rows * ldb, 0.f, C, ldc,
                        s->M * ldc, scales, scales + 1, id, base + offW, planes, nullptr);
    };
    if ((st = launch()) != KT_OK) break;
    (void)hipEventRecord(e0, nullptr);
    for (int r = 0; r < 3 && st == KT_OK; ++r) st = launch();
    (void)hipEventRecord(e1, nullptr);
    if ((e = hipEventSynchronize(e1)) != hipSuccess) { st = hip_fail(h, e, "sync"); break; }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (best < 0 || ms < best_ms) { best = id; best_ms = ms; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != KT_OK) return st;
  if (best < 0) return fail(h, KT_EUNSUPPORTED, "no candidate configuration compiled for this layout");
  *out = best;
  return KT_OK;
}

// Exhaustive selection: every kernel of the dtype (configurations and split-K
// variants), cached per shape.
static kt_status exhaustive_select(Ctx* h, int dtype, const kt_shape* s, int32_t* out) {
  SelState& S = h->sel[dtype];
  const ShapeKey key{s->M, s->N, s->K, s->batch, s->transA, s->transB, dtype};
  auto it = S.exhaustive_cache.find(key);
  if (it != S.exhaustive_cache.end()) { *out = it->second; return KT_OK; }
  std::vector<int32_t> all(num_kernels(h, dtype));
  std::iota(all.begin(), all.end(), 0);
  kt_status st = time_candidates(h, dtype, s, all, out);
  if (st == KT_OK) S.exhaustive_cache[key] = *out;
  return st;
}

static bool outside_box(const SelState& S, const kt_shape& s) {
  const int64_t v[4] = {s.M, s.N, s.K, s.batch};
  for (int f = 0; f < 4; ++f)
    if (v[f] < S.box_lo[f] || v[f] > S.box_hi[f]) return true;
  return false;
}

static void set_box(SelState& S, const kt_shape* shapes, int32_t n) {
  S.have_box = n > 0;
  for (int32_t i = 0; i < n; ++i) {
    const int64_t v[4] = {shapes[i].M, shapes[i].N, shapes[i].K, shapes[i].batch};
    for (int f = 0; f < 4; ++f) {
      if (i == 0 || v[f] < S.box_lo[f]) S.box_lo[f] = v[f];
      if (i == 0 || v[f] > S.box_hi[f]) S.box_hi[f] = v[f];
    }
  }
}

// Fallback for a shape outside the training box: the fastest of the chosen
// kernels and of the split-K variants of their configurations (code the
// deployed set already holds), timed once and cached.
static kt_status fallback_select(Ctx* h, int dtype, const kt_shape* s, int32_t* out) {
  SelState& S = h->sel[dtype];
  const ShapeKey key{s->M, s->N, s->K, s->batch, s->transA, s->transB, dtype};
  auto it = S.fallback_cache.find(key);
  if (it != S.fallback_cache.end()) { *out = it->second; return KT_OK; }
  std::vector<int32_t> cands = S.chosen;
  const int32_t nc = (int32_t)h->configs[dtype].size();
  for (int32_t v = nc; v < num_kernels(h, dtype); ++v) {
    const int32_t b = kernel_base(h, dtype, v);
    bool have_base = false;
    for (int32_t c : S.chosen) have_base = have_base || kernel_base(h, dtype, c) == b;
    if (have_base && std::find(cands.begin(), cands.end(), v) == cands.end()) cands.push_back(v);
  }
  kt_status st = time_candidates(h, dtype, s, cands, out);
  if (st == KT_OK) S.fallback_cache[key] = *out;
  return st;
}



// The fitted model's pick, never the fallback.
static kt_status model_select(Ctx* h, int dtype, const kt_shape* s, int32_t* id) {
  SelState& S = h->sel[dtype];
  switch (S.kind) {
    case KT_SEL_DT_A:
    case KT_SEL_DT_B:
    case KT_SEL_DT_C: {
      const int32_t c = tree_walk(S.tree, *s);
      *id = S.chosen[c];
      return KT_OK;
    }
    case KT_SEL_MLP:
      return mlp_select_host(h, dtype, s, id);
    case KT_SEL_EXHAUSTIVE:
      return exhaustive_select(h, dtype, s, id);
    default:
      return fail(h, KT_ENOTFITTED, "no selector fitted or loaded for this dtype");
  }
}

kt_status select_config(Ctx* h, int dtype, const kt_shape* s, int32_t* id) {
  const SelState& S = h->sel[dtype];
  // Outside the training box the model is extrapolating: time the chosen
  // configurations once instead (not from an entry point that must not
  // allocate, where the model's pick stands).
  if (S.kind >= KT_SEL_DT_A && S.kind <= KT_SEL_MLP && S.fallback && S.have_box &&
      outside_box(S, *s) && !h->forbid_alloc && h->device >= 0)
    return S.fallback == 2 ? exhaustive_select(h, dtype, s, id) : fallback_select(h, dtype, s, id);
  return model_select(h, dtype, s, id);
}

static bool bad_dtype(int d) { return d < 0 || d >= NUM_DTYPES; }

}  // namespace kt

using namespace kt;

extern "C" {

kt_status kt_fit_selector(kt_handle hh, kt_dtype dtype, kt_selector sel, const kt_shape* shapes,
                          const int64_t* time_ns, int32_t n, int32_t d, const int32_t* chosen,
                          int32_t k, const kt_mlp_opts* mlp, void* ws, size_t ws_bytes,
                          void* stream) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (bad_dtype(dtype)) return fail(h, KT_EINVAL, "bad dtype");
  SelState& S = h->sel[dtype];
  if (sel == KT_SEL_EXHAUSTIVE) {
    free_selector_device(h, dtype);
    S = SelState();
    S.kind = KT_SEL_EXHAUSTIVE;
    return KT_OK;
  }
  if ((int)sel < 0 || (int)sel > KT_SEL_MLP) return fail(h, KT_EINVAL, "bad selector kind");
  if (n < 1 || d < 1 || !shapes || !time_ns || !chosen || k < 1 || k > d)
    return fail(h, KT_EINVAL, "bad training data");
  for (int32_t j = 0; j < k; ++j) {
    if (chosen[j] < 0 || chosen[j] >= d || !valid_kernel(h, dtype, chosen[j]))
      return fail(h, KT_EINVAL, "chosen id out of range");
    for (int32_t q = 0; q < j; ++q)
      if (chosen[q] == chosen[j]) return fail(h, KT_EINVAL, "chosen ids must be distinct");
  }
  const int32_t keep_fallback = S.fallback;
  if (sel == KT_SEL_MLP) {
    kt_status st = fit_mlp(h, dtype, shapes, time_ns, n, d, chosen, k, mlp, ws, ws_bytes,
                           (hipStream_t)stream);
    if (st != KT_OK) return st;
    S.fallback = keep_fallback;
    S.kind = KT_SEL_MLP;
    S.tree = Tree();
    S.exhaustive_cache.clear();
    set_box(S, shapes, n);
    return KT_OK;
  }
  CartData D;
  D.n_classes = k;
  D.max_depth = sel == KT_SEL_DT_A ? -1 : sel == KT_SEL_DT_B ? 6 : 3;
  D.min_leaf = sel == KT_SEL_DT_A ? 1 : sel == KT_SEL_DT_B ? 3 : 4;
  D.X.resize(n);
  D.y.resize(n);
  for (int32_t i = 0; i < n; ++i) {
    for (int f = 0; f < 6; ++f) D.X[i][f] = feat(shapes[i], f);
    // label: fastest chosen configuration, lowest position on equal times;
    // non-positive (unmeasured) times never win
    int32_t bj = 0;
    int64_t bt = INT64_MAX;
    for (int32_t j = 0; j < k; ++j) {
      int64_t t = time_ns[(int64_t)i * d + chosen[j]];
      if (t <= 0) t = INT64_MAX;
      if (t < bt) { bt = t; bj = j; }
    }
    D.y[i] = bj;
  }
  Tree T;
  std::vector<int32_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  cart_build(D, idx, 0, T);
  free_selector_device(h, dtype);
  S = SelState();
  S.tree = std::move(T);
  S.chosen.assign(chosen, chosen + k);
  S.kind = sel;
  S.fallback = keep_fallback;
  set_box(S, shapes, n);
  return upload_tree(h, dtype);
}

kt_status kt_select(kt_handle hh, kt_dtype dtype, const kt_shape* s, int32_t* config_id) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (bad_dtype(dtype)) return fail(h, KT_EINVAL, "bad dtype");
  if (!s || !config_id) return fail(h, KT_EINVAL, "NULL argument");
  if (s->M < 0 || s->N < 0 || s->K < 0 || s->batch < 0 || (s->transA & ~1) || (s->transB & ~1))
    return fail(h, KT_EINVAL, "bad shape");
  return select_config(h, dtype, s, config_id);
}

kt_status kt_select_batch(kt_handle hh, kt_dtype dtype, const kt_shape* d_shapes, int32_t n,
                          int32_t* d_ids, void* stream) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (bad_dtype(dtype)) return fail(h, KT_EINVAL, "bad dtype");
  if (!need_device(h)) return KT_EINVAL;
  if (n < 0) return fail(h, KT_EINVAL, "n < 0");
  if (n == 0) return KT_OK;
  if (!d_shapes || !d_ids) return fail(h, KT_EINVAL, "NULL argument");
  SelState& S = h->sel[dtype];
  hipStream_t st = (hipStream_t)stream;
  if (S.kind >= KT_SEL_DT_A && S.kind <= KT_SEL_DT_C) {
    if (!S.d_tree) return fail(h, KT_ENOTFITTED, "tree not on the device");
    hipLaunchKernelGGL(select_tree_kernel, dim3((n + 255) / 256), dim3(256), 0, st, d_shapes, n,
                       (const char*)S.d_tree, (int32_t)S.tree.feature.size(),
                       (int32_t)S.chosen.size(), d_ids);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "select launch");
    return KT_OK;
  }
  if (S.kind == KT_SEL_MLP) return mlp_select_batch(h, dtype, d_shapes, n, d_ids, st);
  if (S.kind == KT_SEL_EXHAUSTIVE)
    return fail(h, KT_EUNSUPPORTED, "exhaustive selection runs per shape on the host (kt_select)");
  return fail(h, KT_ENOTFITTED, "no selector fitted or loaded for this dtype");
}

kt_status kt_get_tree(kt_handle hh, kt_dtype dtype, int32_t* n_nodes, int32_t* feature,
                      int64_t* threshold, int32_t* left, int32_t* right, int32_t* cls) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (bad_dtype(dtype)) return fail(h, KT_EINVAL, "bad dtype");
  if (!n_nodes) return fail(h, KT_EINVAL, "NULL n_nodes");
  const SelState& S = h->sel[dtype];
  if (S.kind < KT_SEL_DT_A || S.kind > KT_SEL_DT_C) return fail(h, KT_ENOTFITTED, "no tree fitted");
  const size_t nn = S.tree.feature.size();
  *n_nodes = (int32_t)nn;
  if (feature) memcpy(feature, S.tree.feature.data(), nn * 4);
  if (threshold) memcpy(threshold, S.tree.threshold.data(), nn * 8);
  if (left) memcpy(left, S.tree.left.data(), nn * 4);
  if (right) memcpy(right, S.tree.right.data(), nn * 4);
  if (cls) memcpy(cls, S.tree.cls.data(), nn * 4);
  return KT_OK;
}

// Text format (version 3; version 2 files, without the box line, load with
// no training box):
//   KTSEL 3
//   selectors <count>
//   then per selector:
//     dtype <d> kind <k>
//     chosen <k> id...
//     tree <n>        followed by n lines: feature threshold left right cls
//     mlp <count>     followed by count floats in %a notation
//     box <have> <fallback> lo_M lo_N lo_K lo_batch hi_M hi_N hi_K hi_batch
//   end
kt_status kt_save(kt_handle hh, const char* path) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!path) return fail(h, KT_EINVAL, "NULL path");
  int count = 0;
  for (int d = 0; d < NUM_DTYPES; ++d) count += h->sel[d].kind >= 0;
  if (count == 0) return fail(h, KT_ENOTFITTED, "nothing to save");
  FILE* f = fopen(path, "w");
  if (!f) return fail(h, KT_EIO, std::string("cannot write ") + path);
  fprintf(f, "KTSEL 3\nselectors %d\n", count);
  for (int d = 0; d < NUM_DTYPES; ++d) {
    const SelState& S = h->sel[d];
    if (S.kind < 0) continue;
    fprintf(f, "dtype %d kind %d\nchosen %zu", d, S.kind, S.chosen.size());
    for (int32_t c : S.chosen) fprintf(f, " %d", c);
    fprintf(f, "\ntree %zu\n", S.tree.feature.size());
    for (size_t i = 0; i < S.tree.feature.size(); ++i)
      fprintf(f, "%d %lld %d %d %d\n", S.tree.feature[i], (long long)S.tree.threshold[i],
              S.tree.left[i], S.tree.right[i], S.tree.cls[i]);
    fprintf(f, "mlp %zu\n", S.mlp.params.size());
    for (float v : S.mlp.params) fprintf(f, "%a\n", (double)v);
    fprintf(f, "box %d %d", S.have_box ? 1 : 0, S.fallback);
    for (int q = 0; q < 4; ++q) fprintf(f, " %lld", (long long)S.box_lo[q]);
    for (int q = 0; q < 4; ++q) fprintf(f, " %lld", (long long)S.box_hi[q]);
    fprintf(f, "\n");
  }
  fprintf(f, "end\n");
  const bool ok = fflush(f) == 0 && !ferror(f);
  fclose(f);
  if (!ok) return fail(h, KT_EIO, std::string("write error on ") + path);
  return KT_OK;
}

kt_status kt_load(kt_handle hh, const char* path) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!path) return fail(h, KT_EINVAL, "NULL path");
  std::ifstream in(path);
  if (!in) return fail(h, KT_EIO, std::string("cannot read ") + path);
  auto bad = [&](const char* why) { return fail(h, KT_EIO, std::string("malformed selector file: ") + why); };
  std::string tag;
  int ver = 0, count = 0;
  if (!(in >> tag >> ver) || tag != "KTSEL" || (ver != 2 && ver != 3)) return bad("header");
  if (!(in >> tag >> count) || tag != "selectors" || count < 1 || count > NUM_DTYPES) return bad("selector count");
  struct Loaded {
    int dtype, kind;
    std::vector<int32_t> chosen;
    Tree tree;
    std::vector<float> params;
    int have_box = 0, fallback = 1;
    long long lo[4] = {0, 0, 0, 0}, hi[4] = {0, 0, 0, 0};
  };
  std::vector<Loaded> all;
  for (int q = 0; q < count; ++q) {
    Loaded L;
    if (!(in >> tag >> L.dtype) || tag != "dtype" || bad_dtype(L.dtype)) return bad("dtype");
    for (const Loaded& o : all) if (o.dtype == L.dtype) return bad("duplicate dtype");
    if (!(in >> tag >> L.kind) || tag != "kind" || L.kind < KT_SEL_DT_A || L.kind > KT_SEL_EXHAUSTIVE) return bad("kind");
    size_t k = 0;
    if (!(in >> tag >> k) || tag != "chosen" || k > 4096) return bad("chosen");
    L.chosen.resize(k);
    for (size_t j = 0; j < k; ++j)
      if (!(in >> L.chosen[j]) || !valid_kernel(h, L.dtype, L.chosen[j]))
        return bad("chosen id");
    size_t nn = 0;
    if (!(in >> tag >> nn) || tag != "tree" || nn > (1u << 24)) return bad("tree");
    Tree& T = L.tree;
    T.feature.resize(nn); T.threshold.resize(nn); T.left.resize(nn); T.right.resize(nn); T.cls.resize(nn);
    for (size_t i = 0; i < nn; ++i) {
      long long thr;
      if (!(in >> T.feature[i] >> thr >> T.left[i] >> T.right[i] >> T.cls[i])) return bad("tree node");
      T.threshold[i] = thr;
      if (T.feature[i] < -1 || T.feature[i] > 5) return bad("feature");
      if (T.feature[i] >= 0 && (T.left[i] <= (int32_t)i || T.right[i] <= (int32_t)i ||
                                T.left[i] >= (int32_t)nn || T.right[i] >= (int32_t)nn))
        return bad("child index");
      if (T.cls[i] < 0 || T.cls[i] >= (int32_t)std::max<size_t>(k, 1)) return bad("class");
    }
    size_t np = 0;
    if (!(in >> tag >> np) || tag != "mlp" || np > (1u << 24)) return bad("mlp");
    L.params.resize(np);
    for (size_t i = 0; i < np; ++i) {
      std::string tok;
      if (!(in >> tok)) return bad("mlp value");
      char* endp = nullptr;
      const double v = strtod(tok.c_str(), &endp);
      if (!endp || *endp) return bad("mlp value");
      L.params[i] = (float)v;
    }
    if (ver >= 3) {
      if (!(in >> tag >> L.have_box >> L.fallback) || tag != "box" || (L.have_box & ~1) ||
          L.fallback < 0 || L.fallback > 2)
        return bad("box");
      for (int q = 0; q < 4; ++q) if (!(in >> L.lo[q])) return bad("box bounds");
      for (int q = 0; q < 4; ++q) if (!(in >> L.hi[q])) return bad("box bounds");
    }
    if (L.kind <= KT_SEL_DT_C && (nn == 0 || k == 0)) return bad("tree selector without nodes");
    if (L.kind == KT_SEL_MLP && np != (size_t)64 * 6 + 64 + 64 * 64 + 64 + k * 64 + k) return bad("mlp size");
    all.push_back(std::move(L));
  }
  if (!(in >> tag) || tag != "end") return bad("end");
  for (Loaded& L : all) {
    free_selector_device(h, L.dtype);
    SelState& S = h->sel[L.dtype];
    S = SelState();
    S.kind = L.kind;
    S.chosen = L.chosen;
    S.tree = std::move(L.tree);
    S.mlp.k = (int32_t)L.chosen.size();
    S.mlp.params = std::move(L.params);
    S.have_box = L.have_box != 0;
    S.fallback = L.fallback;
    for (int q = 0; q < 4; ++q) { S.box_lo[q] = L.lo[q]; S.box_hi[q] = L.hi[q]; }
    kt_status st = KT_OK;
    if (S.kind <= KT_SEL_DT_C) st = upload_tree(h, L.dtype);
    else if (S.kind == KT_SEL_MLP) st = mlp_upload(h, L.dtype);
    if (st != KT_OK) return st;
  }
  return KT_OK;
}

kt_status kt_set_fallback(kt_handle hh, kt_dtype dtype, int32_t enabled) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (bad_dtype(dtype)) return fail(h, KT_EINVAL, "bad dtype");
  if (enabled < 0 || enabled > 2) return fail(h, KT_EINVAL, "fallback mode must be 0, 1 or 2");
  h->sel[dtype].fallback = enabled;
  return KT_OK;
}

kt_status kt_selector_info(kt_handle hh, kt_dtype dtype, int32_t* kind, int32_t* k,
                           int32_t* chosen, int64_t* box, int32_t* fallback) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (bad_dtype(dtype)) return fail(h, KT_EINVAL, "bad dtype");
  const SelState& S = h->sel[dtype];
  if (kind) *kind = S.kind;
  if (k) *k = (int32_t)S.chosen.size();
  if (chosen) memcpy(chosen, S.chosen.data(), S.chosen.size() * 4);
  if (box) {
    for (int q = 0; q < 4; ++q) { box[q] = S.have_box ? S.box_lo[q] : 0; box[4 + q] = S.have_box ? S.box_hi[q] : -1; }
  }
  if (fallback) *fallback = S.fallback;
  return KT_OK;
}

kt_status kt_fit_selector_validated(kt_handle hh, kt_dtype dtype, const kt_shape* shapes,
                                    const int64_t* time_ns, int32_t n, int32_t d,
                                    const int32_t* chosen, int32_t k, const uint8_t* is_validation,
                                    const kt_mlp_opts* mlp, void* ws, size_t ws_bytes, void* stream,
                                    int32_t* kind_out, double* scores) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (bad_dtype(dtype)) return fail(h, KT_EINVAL, "bad dtype");
  if (!shapes || !time_ns || !chosen || !is_validation || !kind_out)
    return fail(h, KT_EINVAL, "NULL argument");
  if (n < 2 || d < 1) return fail(h, KT_EINVAL, "bad training data");
  std::vector<kt_shape> fit_s, val_s;
  std::vector<int64_t> fit_t, val_t;
  for (int32_t i = 0; i < n; ++i) {
    const bool v = is_validation[i] != 0;
    (v ? val_s : fit_s).push_back(shapes[i]);
    std::vector<int64_t>& t = v ? val_t : fit_t;
    t.insert(t.end(), time_ns + (size_t)i * d, time_ns + (size_t)(i + 1) * d);
  }
  if (fit_s.empty() || val_s.empty())
    return fail(h, KT_EINVAL, "need at least one fitting row and one validation row");
  const int32_t nv = (int32_t)val_s.size();
  double best = -1.0;
  int32_t best_kind = -1;
  std::vector<int32_t> picks(nv);
  for (int kind = KT_SEL_DT_A; kind <= KT_SEL_MLP; ++kind) {
    if (kind == KT_SEL_MLP && h->device < 0) {   // a host handle cannot train the MLP
      if (scores) scores[kind] = 0.0;
      continue;
    }
    kt_status st = kt_fit_selector(hh, dtype, (kt_selector)kind, fit_s.data(), fit_t.data(),
                                   (int32_t)fit_s.size(), d, chosen, k, mlp, ws, ws_bytes, stream);
    if (st != KT_OK) return st;
    for (int32_t e = 0; e < nv; ++e)
      if ((st = model_select(h, dtype, &val_s[e], &picks[e])) != KT_OK) return st;
    double log_sum = 0.0;
    for (int32_t e = 0; e < nv; ++e) {
      const int64_t* t = &val_t[(size_t)e * d];
      int64_t tb = 0;
      for (int32_t j = 0; j < d; ++j)
        if (t[j] > 0 && (tb == 0 || t[j] < tb)) tb = t[j];
      const int64_t tu = t[picks[e]];
      if (tb <= 0 || tu <= 0) return fail(h, KT_EINVAL, "validation row without a measured time");
      log_sum += log((double)tb / (double)tu);
    }
    const double score = exp(log_sum / nv);
    if (scores) scores[kind] = score;
    if (score > best) { best = score; best_kind = kind; }
  }
  *kind_out = best_kind;
  return kt_fit_selector(hh, dtype, (kt_selector)best_kind, shapes, time_ns, n, d, chosen, k, mlp,
                         ws, ws_bytes, stream);
}

}  // extern "C"
