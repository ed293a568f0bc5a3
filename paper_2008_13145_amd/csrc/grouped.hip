// Persistent grouped BF16 GEMM: many uneven GEMMs in one launch, captured in
// a hipGraph, with a tile schedule chosen by the library's own autotuner.
//
// The host flattens every member GEMM into output tiles (gemm, tile row,
// tile column, tile class) in a chosen order -- as given, or longest-
// processing-time first (largest K) -- and uploads the member descriptors
// and the work list.  Members with M * N at most a threshold take a smaller
// tile than the rest (the two tiles of a kernel have the same number of
// waves), so small members are not padded out to the large tile.  A grid of
// (#CUs x work-groups per CU) persistent work-groups then walks the list:
// statically (work-group b takes items b, b + grid, ...) or dynamically (an
// atomic counter hands out the next item; a one-thread kernel resets it
// inside the same graph).  Each item runs a BF16 tile of the single-GEMM
// family (A row-major M x K, B row-major K x N, FP32 C): through LDS DMA when
// both member operands have rows on 16-byte boundaries (their rows are then
// read up to the next 16-byte boundary, within the leading dimension), else
// register-staged.
//
// The autotuner searches (tile pair, small-member threshold, schedule,
// order, work-groups per CU) by successive halving on the real workload:
// every candidate's graph is timed, the faster half kept, the repetitions
// doubled, until one remains.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "gemm_lp_dma.hpp"
#include "kt_internal.hpp"

namespace kt {

struct GroupDesc {
  const void* A;
  const void* B;
  float* C;
  int64_t M, N, K, lda, ldb, ldc;
  int32_t vecA, vecB;   // register-path alignment modes
  int32_t dma, pad;     // 1: both operands take the DMA pipeline
};

struct WorkItem {
  int32_t g, tm, tn, cls;   // cls 0: the large tile, 1: the small tile
};

// One tile class.  MODE 0: every member register-staged (the smaller LDS
// footprint keeps more work-groups resident); 1: every member through LDS
// DMA; 2: each member by its own operands (both pipelines compiled into the
// kernel).  The plan picks the mode from its members, and a kernel holds the
// small tile class only when the plan uses it: every tile body compiled into
// the persistent loop keeps its lane-invariant addresses live across the
// whole loop, and with four bodies the kernels ran out of registers.
template <int BM, int BN, int T, int BK, int MODE>
struct GroupTile {
  static constexpr int NT = BM * BN / (T * T);
  static constexpr int L1 = MODE != 1 ? GemmLpCfg<2, BM, BN, T, BK, 0, 0>::LDS_BYTES : 0;
  static constexpr int L2 = MODE != 0 ? LpDmaCfg<2, BM, BN, T, BK, 0, 0>::LDS_BYTES : 0;
  static constexpr int LDS = L1 > L2 ? L1 : L2;

  __device__ __forceinline__ static void run(const GemmArgs& a, int tm, int tn, bool dma,
                                             char* lds) {
    if constexpr (MODE == 1) {
      lp_dma_tile<2, BM, BN, T, BK, 0, 0>(a, tm, tn, 0, lds);
    } else if constexpr (MODE == 2) {
      if (dma) lp_dma_tile<2, BM, BN, T, BK, 0, 0>(a, tm, tn, 0, lds);
      else lp_tile<2, BM, BN, T, BK, 0, 0>(a, tm, tn, 0, reinterpret_cast<uint16_t*>(lds));
    } else {
      lp_tile<2, BM, BN, T, BK, 0, 0>(a, tm, tn, 0, reinterpret_cast<uint16_t*>(lds));
    }
  }
};

// Occupancy target of the DMA-only kernels with one tile class: the waves
// per SIMD that the LDS allows, capped at 2, so a second work-group stays
// resident wherever the LDS has room for it (these kernels fit that register
// budget without spilling; the others do not and keep the compiler's choice).
template <int LDS, int NT, int MODE, bool TWO>
struct GroupOcc {
  static constexpr int RAW = (160 * 1024 / LDS) * (NT / 64) / 4;
  static constexpr int V = (MODE != 1 || TWO) ? 1 : (RAW < 1 ? 1 : (RAW > 2 ? 2 : RAW));
};

template <int BM, int BN, int T, int BK, int SM, int SN, int ST, int SK, int MODE, bool TWO>
__global__ void __launch_bounds__(BM * BN / (T * T))
__attribute__((amdgpu_waves_per_eu(
    GroupOcc<(!TWO || GroupTile<BM, BN, T, BK, MODE>::LDS > GroupTile<SM, SN, ST, SK, MODE>::LDS)
                 ? GroupTile<BM, BN, T, BK, MODE>::LDS
                 : GroupTile<SM, SN, ST, SK, MODE>::LDS,
             BM * BN / (T * T), MODE, TWO>::V,
    8)))
grouped_bf16_kernel(const GroupDesc* __restrict__ descs, const WorkItem* __restrict__ work,
                    int32_t n_work, float alpha, float beta, int32_t dynamic,
                    uint32_t* __restrict__ counter, uint32_t* __restrict__ visits) {
  using Big = GroupTile<BM, BN, T, BK, MODE>;
  using Small = GroupTile<SM, SN, ST, SK, MODE>;
  static_assert(Big::NT == Small::NT, "both tiles of a grouped kernel have the same waves");
  constexpr int LDS = (!TWO || Big::LDS > Small::LDS) ? Big::LDS : Small::LDS;
  __shared__ __attribute__((aligned(16))) char lds[LDS];
  __shared__ int32_t s_w;
  int32_t w = blockIdx.x;
  for (;;) {
    if (dynamic) {
      if (threadIdx.x == 0) s_w = (int32_t)atomicAdd(counter, 1u);
      __syncthreads();
      w = s_w;
    }
    if (w >= n_work) break;
    const WorkItem it = work[w];
    const GroupDesc d = descs[it.g];
    GemmArgs a;
    a.M = d.M; a.N = d.N; a.K = d.K; a.batch = 1;
    a.A = d.A; a.lda = d.lda; a.sA = 0;
    a.B = d.B; a.ldb = d.ldb; a.sB = 0;
    a.C = d.C; a.ldc = d.ldc; a.sC = 0;
    a.alpha = alpha; a.beta = beta;
    a.scaleA = nullptr; a.scaleB = nullptr;
    a.vecA = d.vecA; a.vecB = d.vecB;
    a.tiles_m = 0; a.tiles_n = 0;
    if constexpr (TWO) {
      if (it.cls == 0) Big::run(a, it.tm, it.tn, d.dma != 0, lds);
      else Small::run(a, it.tm, it.tn, d.dma != 0, lds);
    } else {
      Big::run(a, it.tm, it.tn, d.dma != 0, lds);
    }
    if (visits && threadIdx.x == 0) atomicAdd(&visits[w], 1u);
    __syncthreads();   // LDS and s_w are reused by the next item
    if (!dynamic) w += gridDim.x;
  }
}

__global__ void reset_counter_kernel(uint32_t* c) { *c = 0u; }

typedef void (*GroupedKernel)(const GroupDesc*, const WorkItem*, int32_t, float, float, int32_t,
                              uint32_t*, uint32_t*);

struct GroupedVariant {
  int bm, bn, t, bk;       // large tile
  int sm, sn, st, sk;      // small tile (same waves)
  GroupedKernel fn[3][2];  // [mode: register / DMA / per member][small tile class compiled in]
};

#define KT_GK(a, b, c, d, e, f, g, h, m) \
  {grouped_bf16_kernel<a, b, c, d, e, f, g, h, m, false>, grouped_bf16_kernel<a, b, c, d, e, f, g, h, m, true>}
#define KT_GV(a, b, c, d, e, f, g, h) \
  {a, b, c, d, e, f, g, h, {KT_GK(a, b, c, d, e, f, g, h, 0), KT_GK(a, b, c, d, e, f, g, h, 1), \
                            KT_GK(a, b, c, d, e, f, g, h, 2)}}
// Tile pairs the grouped kernel is compiled for (members of the BF16
// configuration space).
static const GroupedVariant kGroupedVariants[] = {
    KT_GV(128, 128, 8, 64, 64, 64, 4, 64),
    KT_GV(128, 128, 8, 32, 64, 64, 4, 32),
    KT_GV(256, 128, 8, 32, 128, 64, 4, 32),
    KT_GV(128, 256, 8, 32, 64, 128, 4, 32),
    KT_GV(256, 256, 8, 64, 128, 128, 4, 64),
    KT_GV(64, 64, 4, 64, 32, 32, 2, 64),
};
#undef KT_GV
#undef KT_GK
static constexpr int kNumVariants = sizeof(kGroupedVariants) / sizeof(kGroupedVariants[0]);

static int32_t config_id_of(Ctx* h, int bm, int bn, int t, int bk) {
  for (int32_t i = 0; i < (int32_t)h->configs[KT_BF16].size(); ++i) {
    const ConfigDef& c = h->configs[KT_BF16][i];
    if (c.bm == bm && c.bn == bn && c.t == t && c.bk == bk) return i;
  }
  return -1;
}

// The compiled pair for (large, small) configuration ids; small -1 matches
// any pair with that large tile (the small tile then goes unused).
static const GroupedVariant* variant_for(Ctx* h, int32_t big, int32_t small) {
  const int32_t n = (int32_t)h->configs[KT_BF16].size();
  if (big < 0 || big >= n || small < -1 || small >= n) return nullptr;
  for (int i = 0; i < kNumVariants; ++i) {
    const GroupedVariant& v = kGroupedVariants[i];
    if (config_id_of(h, v.bm, v.bn, v.t, v.bk) != big) continue;
    if (small < 0 || config_id_of(h, v.sm, v.sn, v.st, v.sk) == small) return &v;
  }
  return nullptr;
}

static size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

// Smallest tile of any variant (32 x 32) bounds the work list length.
static int64_t max_work_items(const kt_shape* s, int32_t n) {
  int64_t tot = 0;
  for (int32_t i = 0; i < n; ++i) tot += cdiv(s[i].M, 32) * cdiv(s[i].N, 32);
  return tot;
}

}  // namespace kt

struct kt_grouped_plan_s {
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  int32_t n_work = 0;
  kt_grouped_opts opts;
};

using namespace kt;

namespace kt {

static kt_status validate_group(Ctx* h, kt_dtype dtype, const kt_shape* shapes, int32_t n,
                                const void* const* A, const void* const* B, float* const* C,
                                const int64_t* ld) {
  if (dtype != KT_BF16) return fail(h, KT_EUNSUPPORTED, "grouped GEMM supports BF16 inputs");
  if (n < 0 || (n > 0 && (!shapes || !A || !B || !C))) return fail(h, KT_EINVAL, "bad group arrays");
  for (int32_t i = 0; i < n; ++i) {
    const kt_shape& s = shapes[i];
    if (s.M < 0 || s.N < 0 || s.K < 0) return fail(h, KT_EINVAL, "negative size in group");
    if (s.batch != 1 || s.transA != 0 || s.transB != 0)
      return fail(h, KT_EUNSUPPORTED, "grouped members must be batch 1, transA = transB = 0");
    if (s.M > 0 && s.N > 0 && (!C[i] || (s.K > 0 && (!A[i] || !B[i]))))
      return fail(h, KT_EINVAL, "NULL member pointer");
    if (ld && (ld[3 * i] < std::max<int64_t>(s.K, 1) || ld[3 * i + 1] < std::max<int64_t>(s.N, 1) ||
               ld[3 * i + 2] < std::max<int64_t>(s.N, 1)))
      return fail(h, KT_EINVAL, "member leading dimension below its row length");
  }
  return KT_OK;
}

// Member operand alignment: the register pipeline's mode and whether the
// DMA pipeline may read the operand (rows on 16-byte boundaries and the row's
// last 16-byte chunk within the leading dimension: member rows are allocated
// in full, so reading up to the next 16-byte boundary stays inside them).
static int32_t member_vec(const void* p, int64_t ld) {
  if ((uintptr_t)p % 4 != 0) return LP_ALIGN_NONE;
  return ld % 2 == 0 ? LP_ALIGN_ROWS : LP_ALIGN_BASE;
}
static bool member_dma(const void* p, int64_t ld, int64_t ext) {
  return (uintptr_t)p % 16 == 0 && ld % 8 == 0 && ext >= 8 && ld >= (ext + 7) / 8 * 8;
}

// XCD-blocked tile order of one member: its tile grid cut into 8 rectangles
// (r rows x c columns of blocks, r c = 8, the blocks as square as the grid
// allows), emitted interleaved -- block x's j-th tile at position 8 j + x of
// the member's run -- so that round-robin dispatch over the 8 XCDs gives each
// XCD one rectangle and its L2 serves the A and B panels the rectangle's
// tiles share.  False (nothing emitted) for grids too small to cut.
static bool blocked_tiles(int32_t g, int tmn, int tnn, int cls, std::vector<WorkItem>& work) {
  int best_r = 0;
  double best = 0.0;
  for (int r = 1; r <= 8; r *= 2) {
    const int c = 8 / r;
    if (tmn < r || tnn < c) continue;
    const double bh = (double)tmn / r, bw = (double)tnn / c;
    const double score = std::min(bh, bw) / std::max(bh, bw);
    if (best_r == 0 || score > best) { best_r = r; best = score; }
  }
  if (best_r == 0) return false;
  const int r = best_r, c = 8 / r;
  std::vector<std::vector<WorkItem>> blocks(8);
  for (int bi = 0; bi < r; ++bi)
    for (int bj = 0; bj < c; ++bj) {
      std::vector<WorkItem>& b = blocks[bi * c + bj];
      for (int tm = (int)((int64_t)tmn * bi / r); tm < (int)((int64_t)tmn * (bi + 1) / r); ++tm)
        for (int tn = (int)((int64_t)tnn * bj / c); tn < (int)((int64_t)tnn * (bj + 1) / c); ++tn)
          b.push_back(WorkItem{g, tm, tn, cls});
    }
  size_t longest = 0;
  for (const auto& b : blocks) longest = std::max(longest, b.size());
  for (size_t j = 0; j < longest; ++j)
    for (const auto& b : blocks)
      if (j < b.size()) work.push_back(b[j]);
  return true;
}

static kt_status plan_build(Ctx* h, const kt_shape* shapes, int32_t n, const void* const* A,
                            const void* const* B, float* const* C, const int64_t* ld, float alpha,
                            float beta, const kt_grouped_opts& o, void* ws, size_t ws_bytes,
                            hipStream_t stream, kt_grouped_plan_s** out) {
  const GroupedVariant* v = variant_for(h, o.config_id, o.small_config_id);
  if (!v) return fail(h, KT_EUNSUPPORTED, "BF16 tile pair not compiled for the grouped kernel");
  if (o.small_max_area < 0) return fail(h, KT_EINVAL, "negative small-member area");
  if (o.schedule < 0 || o.schedule > 1 || o.order < 0 || o.order > 3 || o.wgs_per_cu < 1 ||
      o.wgs_per_cu > 4 || o.pipeline < 0 || o.pipeline > 1)
    return fail(h, KT_EINVAL, "bad grouped options");
  const size_t need = a256((size_t)n * sizeof(GroupDesc)) + a256((size_t)max_work_items(shapes, n) * sizeof(WorkItem)) + 256;
  if (!ws || ws_bytes < need) return fail(h, KT_EWORKSPACE, "grouped workspace too small");
  std::vector<GroupDesc> descs(n);
  for (int32_t i = 0; i < n; ++i) {
    const kt_shape& s = shapes[i];
    GroupDesc& d = descs[i];
    d.A = A[i]; d.B = B[i]; d.C = C[i];
    d.M = s.M; d.N = s.N; d.K = s.K;
    d.lda = ld ? ld[3 * i] : std::max<int64_t>(s.K, 1);
    d.ldb = ld ? ld[3 * i + 1] : std::max<int64_t>(s.N, 1);
    d.ldc = ld ? ld[3 * i + 2] : std::max<int64_t>(s.N, 1);
    d.vecA = member_vec(A[i], d.lda);
    d.vecB = member_vec(B[i], d.ldb);
    d.dma = o.pipeline == 0 && s.K > 0 && member_dma(A[i], d.lda, s.K) &&
            member_dma(B[i], d.ldb, s.N);
    d.pad = 0;
  }
  std::vector<int32_t> gorder(n);
  std::iota(gorder.begin(), gorder.end(), 0);
  if (o.order & 1)   // longest processing time first: tile work grows with K
    std::stable_sort(gorder.begin(), gorder.end(), [&](int32_t a, int32_t b) { return shapes[a].K > shapes[b].K; });
  std::vector<WorkItem> work;
  for (int32_t g : gorder) {
    const kt_shape& s = shapes[g];
    if (s.M == 0 || s.N == 0) continue;
    const int cls = (o.small_config_id >= 0 && s.M * s.N <= o.small_max_area) ? 1 : 0;
    const int bm = cls ? v->sm : v->bm, bn = cls ? v->sn : v->bn;
    const int tmn = (int)cdiv(s.M, bm), tnn = (int)cdiv(s.N, bn);
    if ((o.order & 2) && blocked_tiles(g, tmn, tnn, cls, work)) continue;
    for (int tm = 0; tm < tmn; ++tm)
      for (int tn = 0; tn < tnn; ++tn) work.push_back(WorkItem{g, tm, tn, cls});
  }
  char* w = (char*)ws;
  GroupDesc* d_desc = (GroupDesc*)w;
  WorkItem* d_work = (WorkItem*)(w + a256((size_t)n * sizeof(GroupDesc)));
  uint32_t* d_counter = (uint32_t*)(w + a256((size_t)n * sizeof(GroupDesc)) +
                                    a256((size_t)max_work_items(shapes, n) * sizeof(WorkItem)));
  hipError_t e = hipSuccess;
  if (n > 0) e = hipMemcpyAsync(d_desc, descs.data(), n * sizeof(GroupDesc), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && !work.empty())
    e = hipMemcpyAsync(d_work, work.data(), work.size() * sizeof(WorkItem), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(h, e, "upload grouped work list");
  hipDeviceProp_t prop;
  if ((e = hipGetDeviceProperties(&prop, h->device)) != hipSuccess) return hip_fail(h, e, "device properties");
  const int n_work = (int)work.size();
  const int grid = std::max(1, std::min(n_work, prop.multiProcessorCount * o.wgs_per_cu));
  const int threads = v->bm * v->bn / (v->t * v->t);
  hipStream_t cs;
  if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) return hip_fail(h, e, "capture stream");
  kt_grouped_plan_s* plan = new kt_grouped_plan_s();
  plan->n_work = n_work;
  plan->opts = o;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess && n_work > 0) {
    if (o.schedule == 1) hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, cs, d_counter);
    // register-staged only, DMA only (every member with work allows it; a
    // member with K = 0 has nothing to load), or per member
    bool any_dma = false, all_dma = true, two = false;
    for (int32_t i = 0; i < n; ++i) {
      if (shapes[i].M == 0 || shapes[i].N == 0) continue;
      any_dma = any_dma || descs[i].dma;
      all_dma = all_dma && (descs[i].dma || shapes[i].K == 0);
    }
    for (const WorkItem& it : work) two = two || it.cls == 1;
    const int mode = !any_dma ? 0 : (all_dma ? 1 : 2);
    hipLaunchKernelGGL(v->fn[mode][two ? 1 : 0], dim3(grid), dim3(threads), 0, cs,
                       (const GroupDesc*)d_desc,
                       (const WorkItem*)d_work, n_work, alpha, beta, (int32_t)o.schedule, d_counter,
                       o.visits);
  }
  hipError_t e2 = hipStreamEndCapture(cs, &plan->graph);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    delete plan;
    return hip_fail(h, e, "grouped graph capture");
  }
  *out = plan;
  return KT_OK;
}

static void plan_free(kt_grouped_plan_s* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  delete p;
}

static kt_grouped_opts default_grouped_opts(Ctx* h) {
  kt_grouped_opts o;
  memset(&o, 0, sizeof o);
  o.config_id = config_id_of(h, 128, 128, 8, 32);
  o.small_config_id = config_id_of(h, 64, 64, 4, 32);
  o.small_max_area = 256 * 256;
  o.schedule = 1;
  o.order = 1;
  o.wgs_per_cu = 2;
  return o;
}

}  // namespace kt

extern "C" {

kt_status kt_grouped_workspace_bytes(const kt_shape* shapes, int32_t n, size_t* bytes) {
  if (!bytes || n < 0 || (n > 0 && !shapes)) return KT_EINVAL;
  *bytes = a256((size_t)n * sizeof(GroupDesc)) + a256((size_t)max_work_items(shapes, n) * sizeof(WorkItem)) + 256;
  return KT_OK;
}

kt_status kt_grouped_num_candidates(int32_t* n) {
  if (!n) return KT_EINVAL;
  *n = kNumVariants;
  return KT_OK;
}

kt_status kt_grouped_plan_create(kt_handle hh, kt_dtype dtype, const kt_shape* shapes, int32_t n,
                                 const void* const* A, const void* const* B, float* const* C,
                                 const int64_t* ld, float alpha, float beta,
                                 const kt_grouped_opts* opts, void* workspace, size_t ws_bytes,
                                 void* stream, kt_grouped_plan* out) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  if (!out) return fail(h, KT_EINVAL, "NULL plan output");
  kt_status s = validate_group(h, dtype, shapes, n, A, B, C, ld);
  if (s != KT_OK) return s;
  kt_grouped_opts o = opts ? *opts : (h->grouped_tuned ? h->grouped_best : default_grouped_opts(h));
  kt_grouped_plan_s* p = nullptr;
  s = plan_build(h, shapes, n, A, B, C, ld, alpha, beta, o, workspace, ws_bytes,
                 (hipStream_t)stream, &p);
  if (s != KT_OK) return s;
  *out = p;
  return KT_OK;
}

kt_status kt_grouped_plan_launch(kt_handle hh, kt_grouped_plan plan, void* stream) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!plan) return fail(h, KT_EINVAL, "NULL plan");
  if (plan->n_work == 0) return KT_OK;
  hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(h, e, "grouped graph launch");
  return KT_OK;
}

kt_status kt_grouped_plan_info(kt_grouped_plan plan, int32_t* n_work, kt_grouped_opts* opts) {
  if (!plan) return KT_EINVAL;
  if (n_work) *n_work = plan->n_work;
  if (opts) *opts = plan->opts;
  return KT_OK;
}

kt_status kt_grouped_plan_destroy(kt_grouped_plan plan) {
  plan_free(plan);
  return KT_OK;
}

kt_status kt_grouped_gemm(kt_handle hh, kt_dtype dtype, const kt_shape* shapes, int32_t n,
                          const void* const* A, const void* const* B, float* const* C,
                          const int64_t* ld, float alpha, float beta, const kt_grouped_opts* opts,
                          void* workspace, size_t ws_bytes, void* stream) {
  kt_grouped_plan p = nullptr;
  kt_status s = kt_grouped_plan_create(hh, dtype, shapes, n, A, B, C, ld, alpha, beta, opts,
                                       workspace, ws_bytes, stream, &p);
  if (s != KT_OK) return s;
  s = kt_grouped_plan_launch(hh, p, stream);
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  plan_free(p);
  if (s == KT_OK && e != hipSuccess) s = hip_fail(h, e, "grouped sync");
  return s;
}

kt_status kt_autotune_grouped(kt_handle hh, kt_dtype dtype, const kt_shape* shapes, int32_t n,
                              const void* const* A, const void* const* B, float* const* C,
                              const int64_t* ld, void* workspace, size_t ws_bytes, void* stream,
                              kt_grouped_opts* best, float* best_ms, int32_t* evaluations) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  kt_status s = validate_group(h, dtype, shapes, n, A, B, C, ld);
  if (s != KT_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  std::vector<kt_grouped_opts> cands;
  static const int64_t kAreas[] = {0, 128 * 128, 256 * 256, 512 * 512};
  // register-staged only, and (where some member allows it) the DMA pipeline
  bool any_dma = false;
  for (int32_t i = 0; i < n && !any_dma; ++i) {
    const int64_t lda = ld ? ld[3 * i] : std::max<int64_t>(shapes[i].K, 1);
    const int64_t ldb = ld ? ld[3 * i + 1] : std::max<int64_t>(shapes[i].N, 1);
    any_dma = shapes[i].K > 0 && member_dma(A[i], lda, shapes[i].K) &&
              member_dma(B[i], ldb, shapes[i].N);
  }
  for (int vi = 0; vi < kNumVariants; ++vi) {
    const GroupedVariant& v = kGroupedVariants[vi];
    const int32_t big = config_id_of(h, v.bm, v.bn, v.t, v.bk);
    const int32_t small = config_id_of(h, v.sm, v.sn, v.st, v.sk);
    if (big < 0 || small < 0) continue;
    for (int64_t area : kAreas)
      for (int sched = 0; sched < 2; ++sched)
        for (int order = 0; order < 4; ++order)
          for (int wgs = 1; wgs <= 2; ++wgs)
            for (int pipe = any_dma ? 0 : 1; pipe < 2; ++pipe) {
              kt_grouped_opts o;
              memset(&o, 0, sizeof o);
              o.config_id = big;
              o.small_config_id = area > 0 ? small : -1;
              o.small_max_area = area;
              o.schedule = sched; o.order = order; o.wgs_per_cu = wgs;
              o.pipeline = pipe;
              cands.push_back(o);
            }
  }
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return hip_fail(h, e, "event");
  if ((e = hipEventCreate(&e1)) != hipSuccess) { (void)hipEventDestroy(e0); return hip_fail(h, e, "event"); }
  std::vector<float> score(cands.size(), 0.f);
  std::vector<int> alive(cands.size());
  std::iota(alive.begin(), alive.end(), 0);
  int reps = 1, evals = 0;
  while (s == KT_OK) {
    for (int ci : alive) {
      kt_grouped_plan_s* p = nullptr;
      s = plan_build(h, shapes, n, A, B, C, ld, 1.f, 0.f, cands[ci], workspace, ws_bytes, st, &p);
      if (s != KT_OK) break;
      e = hipGraphLaunch(p->exec, st);                   // warm-up
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      for (int r = 0; r < reps && e == hipSuccess; ++r) e = hipGraphLaunch(p->exec, st);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      plan_free(p);
      if (e != hipSuccess) { s = hip_fail(h, e, "autotune timing"); break; }
      score[ci] = ms / reps;
      ++evals;
    }
    if (s != KT_OK || alive.size() == 1) break;
    std::stable_sort(alive.begin(), alive.end(), [&](int a, int b) { return score[a] < score[b]; });
    alive.resize((alive.size() + 1) / 2);
    reps *= 2;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != KT_OK) return s;
  h->grouped_best = cands[alive[0]];
  h->grouped_tuned = true;
  if (best) *best = cands[alive[0]];
  if (best_ms) *best_ms = score[alive[0]];
  if (evaluations) *evaluations = evals;
  return KT_OK;
}

}  // extern "C"
