// Direct-to-LDS pipeline of the low-precision family, taken when every
// operand row starts on a 16-byte boundary (base, leading dimension and
// batch stride multiples of 16 bytes) and no 16-byte chunk read can leave
// the operand: its contiguous extent (K, or M / N for an operand stored M- /
// N-contiguous) is whole chunks, or (grouped members, whose rows are
// allocated to the full leading dimension) the last chunk of a row ends
// within the leading dimension.  Same configuration knobs and results
// contract as gemm_lp.hpp; what changes is how tiles reach the MFMAs:
//
// * Global -> LDS with gfx950's 16-byte LDS DMA (global_load_lds_dwordx4):
//   each wave instruction moves 1 KiB straight into LDS (lane l's 16 bytes
//   land at the instruction's LDS base + 16 l), with no register staging, so
//   NS stages (2..4, as many as the LDS budget allows) are in flight at once
//   and a stage is waited for with vmcnt, not refetched through VGPRs.
// * An operand stored with K contiguous keeps that layout in LDS ([row][k],
//   rows of BK elements); its MFMA fragments are 16-byte LDS reads.  The
//   16-byte chunks of a row are XOR-swizzled by the row index so that the 16
//   rows one read phase touches fall on distinct bank groups.
// * An operand stored with M (or N) contiguous is copied as stored
//   ([k][col]) and its fragments come from the LDS transpose reads
//   (ds_read_b64_tr_b16 for BF16: lane j of a 16-lane group receives four
//   consecutive k of column j from the 4 x 16 block the group addresses;
//   ds_read_b64_tr_b8 for FP8: eight consecutive k of column j from an
//   8 x 16 block), chunks swizzled by k so the rows read together spread
//   over the banks.
// * Out-of-range rows and columns are read from clamped in-range addresses
//   (those outputs are never stored); K beyond the product in the last stage
//   is zeroed in LDS after it lands, so it adds nothing.
#pragma once
#include "gemm_lp.hpp"

namespace kt {

// GemmArgs::vecA / vecB value for rows on 16-byte boundaries.
enum { LP_ALIGN_DMA = 3 };

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void gbl_void_t;
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef int i32x2 __attribute__((ext_vector_type(2)));

// Wait until at most N of this wave's vector-memory operations (the LDS DMA
// of later stages) are outstanding and its LDS reads have returned, then
// meet the other waves.  One asm block, so nothing is moved across it.
template <int N>
__device__ __forceinline__ void vm_wait_barrier() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  asm volatile("s_waitcnt vmcnt(%0)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" ::"n"(N) : "memory");
}

// One lane's 16 bytes of a wave's 1 KiB LDS DMA: global `src` to the LDS
// block at `dst` (wave-uniform; lane l's bytes land at dst + 16 l).  Written
// as inline asm so the compiler does not track it: its waitcnt pass cannot
// tell which stage buffer a transpose read touches and otherwise waits for
// every DMA in flight -- the next stage's included -- before each stage's
// fragment reads.  Every wait on these transfers is the explicit one of the
// stage pipeline (vm_wait_barrier); vector-memory operations complete in
// issue order, so the compiler's own vmcnt waits stay correct.
__device__ __forceinline__ void lds_dma16(const void* src, void* dst) {
  const uint32_t m0 = __builtin_amdgcn_readfirstlane(
      (uint32_t)(uintptr_t)(lds_void_t*)dst);
  asm volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src), "{m0}"(m0));
}

template <int EB, int BM, int BN, int T, int BK, int TA, int TB>
struct LpDmaCfg {
  using Base = GemmLpCfg<EB, BM, BN, T, BK, TA, TB>;
  static constexpr int NT = Base::NT, WAVES = Base::WAVES;
  static constexpr int A_BYTES = BM * BK * EB, B_BYTES = BN * BK * EB;
  static constexpr int STAGE = A_BYTES + B_BYTES;
  // Large tiles run one work-group per CU and take as many stages as fit;
  // smaller ones leave room for a second work-group.
  static constexpr int BUDGET = (BM * BN >= 256 * 128) ? 160 * 1024 : 80 * 1024;
  static constexpr int NS_FIT = BUDGET / STAGE;
  static constexpr int NS = NS_FIT < 2 ? 2 : (NS_FIT > 4 ? 4 : NS_FIT);
  static constexpr int LDS_BYTES = NS * STAGE;
  static constexpr int NBA = A_BYTES / 1024, NBB = B_BYTES / 1024;   // 1 KiB DMA blocks
  static constexpr int NBLK = NBA + NBB;
  static constexpr int NW_LO = NBLK / WAVES, NW_HI = (NBLK + WAVES - 1) / WAVES;
  // Occupancy target: the waves per SIMD that the LDS footprint allows,
  // capped at 2, so the register budget (512 / waves) keeps a second
  // work-group resident wherever the LDS has room for it.
  static constexpr int OCC_LDS = (160 * 1024 / LDS_BYTES) * WAVES / 4;
  static constexpr int OCC = OCC_LDS < 1 ? 1 : (OCC_LDS > 2 ? 2 : OCC_LDS);
  static_assert(A_BYTES % 1024 == 0 && B_BYTES % 1024 == 0, "tiles of whole 1 KiB blocks");
  static_assert(LDS_BYTES <= 160 * 1024, "LDS budget");
  static_assert((NS - 2) * NW_HI < 64, "vmcnt range");
};

// Stage wait: at most `ahead` (0 .. NS - 2) later stages of NW blocks each
// may still be in flight.
template <int NW, int NS>
__device__ __forceinline__ void wait_stage(int ahead) {
  if constexpr (NS >= 4) {
    if (ahead >= 2) { vm_wait_barrier<2 * NW>(); return; }
  }
  if constexpr (NS >= 3) {
    if (ahead >= 1) { vm_wait_barrier<NW>(); return; }
  }
  vm_wait_barrier<0>();
}

// Chunk swizzles.  K-major rows hold CPR 16-byte chunks; chunk c of row r
// sits at c ^ kswz(r): the 16 consecutive rows a fragment read touches land
// on 16 distinct 16-byte bank groups of the 256-byte bank line.
template <int CPR>
__device__ __forceinline__ int kswz(int r) {
  constexpr int RP = CPR >= 16 ? 1 : 16 / CPR;   // rows per 256 bytes
  return (r / RP) % CPR;
}
// MN-major rows (one k each): the rows a transpose read covers together
// (4 for BF16, 8 for FP8, each W = 16 / rows chunks wide) are moved W chunks
// apart per 256-byte line.
template <int CPR, int W>
__device__ __forceinline__ int mswz(int k) {
  constexpr int RP = CPR >= 16 ? 1 : 16 / CPR;
  return ((k / RP) * W) % CPR;
}

// Issue this wave's DMA blocks of one stage.  Block q of the stage (0 ..
// NBA-1: A, then B) is handled by wave q % WAVES.  Rows / columns beyond the
// operand are clamped to in-range addresses.
template <int EB, int BM, int BN, int T, int BK, int TA, int TB>
__device__ __forceinline__ void lp_dma_issue(const GemmArgs& args, const char* __restrict__ Ag,
                                             const char* __restrict__ Bg, int64_t m0, int64_t n0,
                                             int64_t k0, char* stage, int wave, int lane) {
  using Cfg = LpDmaCfg<EB, BM, BN, T, BK, TA, TB>;
  constexpr int CE = 16 / EB;   // elements per chunk
#pragma unroll
  for (int i = 0; i < Cfg::NW_HI; ++i) {
    const int q = wave + i * Cfg::WAVES;
    if (q >= Cfg::NBLK) break;   // wave-uniform
    const bool isA = q < Cfg::NBA;
    const int blk = isA ? q : q - Cfg::NBA;
    const int o = blk * 1024 + lane * 16;   // byte offset in the operand's stage tile
    const bool kmajor = isA ? (TA == 0) : (TB == 1);
    const int rows_c = isA ? BM : BN;        // M or N extent of the tile
    const int64_t lim = isA ? args.M : args.N;
    const int64_t ld = isA ? args.lda : args.ldb;
    const int64_t c0 = isA ? m0 : n0;
    const char* base = isA ? Ag : Bg;
    int64_t elem;   // element offset of the 16-byte chunk in the operand
    if (kmajor) {
      constexpr int ROWB = BK * EB, CPR = ROWB / 16;
      const int r = o / ROWB, p = (o % ROWB) / 16;
      const int c = p ^ kswz<CPR>(r);
      int64_t row = c0 + r;
      row = row < lim ? row : lim - 1;
      int64_t kk = k0 + (int64_t)c * CE;
      kk = kk < args.K ? kk : ((args.K - 1) / CE) * CE;   // chunks beyond K: the last one
      elem = row * ld + kk;
    } else {
      const int ROWB = rows_c * EB, CPR = ROWB / 16;
      const int k = o / ROWB, p = (o % ROWB) / 16;
      const int W = EB == 2 ? 4 : 2;
      const int RP = CPR >= 16 ? 1 : 16 / CPR;
      const int c = p ^ (((k / RP) * W) % CPR);
      int64_t kr = k0 + k;
      kr = kr < args.K ? kr : args.K - 1;
      int64_t col = c0 + (int64_t)c * CE;
      col = col < lim ? col : ((lim - 1) / CE) * CE;      // chunks beyond the extent: the last
      elem = kr * ld + col;
    }
    char* dst = stage + (isA ? 0 : Cfg::A_BYTES) + blk * 1024;
    lds_dma16(base + elem * EB, dst);
  }
}

// Zero K positions kvalid .. BK-1 of a stage (the last, partial one).
template <int EB, int BM, int BN, int T, int BK, int TA, int TB>
__device__ __forceinline__ void lp_dma_zero_tail(char* stage, int kvalid, int tid) {
  using Cfg = LpDmaCfg<EB, BM, BN, T, BK, TA, TB>;
  typedef typename LpElem<EB>::T E;
#pragma unroll
  for (int op = 0; op < 2; ++op) {
    const bool kmajor = op == 0 ? (TA == 0) : (TB == 1);
    const int rows_c = op == 0 ? BM : BN;
    E* t = reinterpret_cast<E*>(stage + (op == 0 ? 0 : Cfg::A_BYTES));
    const int tail = BK - kvalid;
    if (kmajor) {
      constexpr int CPR = BK * EB / 16, CE = 16 / EB;
      for (int i = tid; i < rows_c * tail; i += Cfg::NT) {
        const int r = i / tail, k = kvalid + i % tail;
        const int c = k / CE, w = k % CE;
        t[r * BK + (c ^ kswz<CPR>(r)) * CE + w] = (E)0;
      }
    } else {
      for (int i = tid; i < rows_c * tail; i += Cfg::NT) t[kvalid * rows_c + i] = (E)0;
    }
  }
}

// One lane's MFMA fragment of MFMA block `blk` (rows or columns blk * MB ..)
// for K step s of a stage tile held K-major.
template <int EB, int BK, int MB, int KSTEP>
__device__ __forceinline__ void lp_frag_kmajor(LpFrag<EB>& f, const char* tile, int row, int s,
                                               int kh) {
  constexpr int CPR = BK * EB / 16;
  const int c = (s * KSTEP + kh) * EB / 16;
  const char* rp = tile + row * (BK * EB);
  if constexpr (EB == 2) {
    f.read(rp + (c ^ kswz<CPR>(row)) * 16);
  } else {
    const u32x4 lo = *reinterpret_cast<const u32x4*>(rp + (c ^ kswz<CPR>(row)) * 16);
    const u32x4 hi = *reinterpret_cast<const u32x4*>(rp + ((c + 1) ^ kswz<CPR>(row)) * 16);
    i32x8 v;
    v[0] = lo[0]; v[1] = lo[1]; v[2] = lo[2]; v[3] = lo[3];
    v[4] = hi[0]; v[5] = hi[1]; v[6] = hi[2]; v[7] = hi[3];
    f.v = v;
  }
}

// The same for a tile held MN-major ([k][col], COLS columns): transpose
// reads.  colg is the first column of this lane's 16-lane group, kg its
// first k in the stage.
template <int EB, int COLS>
__device__ __forceinline__ void lp_frag_mnmajor(LpFrag<EB>& f, const char* tile, int colg, int kg,
                                                int j) {
  constexpr int ROWB = COLS * EB, CPR = ROWB / 16;
  if constexpr (EB == 2) {
    // source lane j = 4 r + c reads k row kg + kq + r, columns colg + 4c .. + 3
    const int r = j >> 2, cq = j & 3;
    const int byte = (colg + 4 * cq) * 2;
    s16x4 h[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int k = kg + 4 * q + r;
      const char* p = tile + k * ROWB + (((byte >> 4) ^ mswz<CPR, 4>(k)) << 4) + (byte & 15);
      h[q] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) s16x4*)(p));
    }
    typedef short s16x8 __attribute__((ext_vector_type(8)));
    s16x8 v;
    v[0] = h[0][0]; v[1] = h[0][1]; v[2] = h[0][2]; v[3] = h[0][3];
    v[4] = h[1][0]; v[5] = h[1][1]; v[6] = h[1][2]; v[7] = h[1][3];
    f.v = __builtin_bit_cast(bf16x8, v);
  } else {
    // source lane j = 2 r + c reads k row kg + 8q + r, columns colg + 8c .. + 7
    const int r = j >> 1, cq = j & 1;
    const int byte = colg + 8 * cq;
    i32x8 v;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = kg + 8 * q + r;
      const char* p = tile + k * ROWB + (((byte >> 4) ^ mswz<CPR, 2>(k)) << 4) + (byte & 15);
      const i32x2 w = __builtin_amdgcn_ds_read_tr8_b64_v2i32((__attribute__((address_space(3))) i32x2*)(p));
      v[2 * q] = w[0];
      v[2 * q + 1] = w[1];
    }
    f.v = v;
  }
}

// One BM x BN output tile through the DMA pipeline.  lds holds NS stages;
// the caller synchronizes before reusing it for another tile.
template <int EB, int BM, int BN, int T, int BK, int TA, int TB>
__device__ __forceinline__ void lp_dma_tile(const GemmArgs& args, int tm, int tn, int64_t bz,
                                            char* lds) {
  using Cfg = LpDmaCfg<EB, BM, BN, T, BK, TA, TB>;
  using Base = typename Cfg::Base;
  constexpr int NS = Cfg::NS;
  constexpr int WT = Base::WT, MB = Base::MB, SUB = Base::SUB, KSTEP = Base::KSTEP;
  constexpr int NKK = BK / KSTEP;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave / Base::WAVES_N) * WT;
  const int wn0 = (wave % Base::WAVES_N) * WT;
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int64_t M = args.M, N = args.N, K = args.K;
  const char* __restrict__ Ag = static_cast<const char*>(args.A) + bz * args.sA * EB;
  const char* __restrict__ Bg = static_cast<const char*>(args.B) + bz * args.sB * EB;
  float scale = args.alpha;
  if (EB == 1) scale = args.alpha / (args.scaleA[0] * args.scaleB[0]);

  typedef typename std::conditional<MB == 16, f32x4, f32x16>::type Acc;
  constexpr int NACC = MB == 16 ? 4 : 16;
  Acc acc[SUB][SUB];
#pragma unroll
  for (int i = 0; i < SUB; ++i)
#pragma unroll
    for (int j = 0; j < SUB; ++j)
#pragma unroll
      for (int r = 0; r < NACC; ++r) acc[i][j][r] = 0.f;

  const int rb = lane % MB, kh = (lane / MB) * (KSTEP * MB / 64);
  const int j16 = lane & 15;
  const int gcol = rb - j16;   // first column of this lane's 16-lane group within its block
  const int nk = (int)((K + BK - 1) / BK);
  const int my_blocks = (wave < Cfg::NBLK % Cfg::WAVES || Cfg::NBLK % Cfg::WAVES == 0)
                            ? Cfg::NW_HI : Cfg::NW_LO;

#pragma unroll
  for (int s = 0; s < NS - 1; ++s)
    if (s < nk)
      lp_dma_issue<EB, BM, BN, T, BK, TA, TB>(args, Ag, Bg, m0, n0, (int64_t)s * BK,
                                              lds + s * Cfg::STAGE, wave, lane);

  for (int kt = 0; kt < nk; ++kt) {
    // stage kt has landed once at most `ahead` later stages are in flight
    const int ahead = min(NS - 2, nk - 1 - kt);
    if (my_blocks == Cfg::NW_HI) wait_stage<Cfg::NW_HI, NS>(ahead);
    else wait_stage<Cfg::NW_LO, NS>(ahead);
    char* cur = lds + (kt % NS) * Cfg::STAGE;
    if (kt == nk - 1 && K - (int64_t)kt * BK < BK) {
      lp_dma_zero_tail<EB, BM, BN, T, BK, TA, TB>(cur, (int)(K - (int64_t)kt * BK), tid);
      vm_wait_barrier<0>();
    }
    // the buffer of stage kt - 1 is free: every wave has passed its reads
    if (kt + NS - 1 < nk)
      lp_dma_issue<EB, BM, BN, T, BK, TA, TB>(args, Ag, Bg, m0, n0, (int64_t)(kt + NS - 1) * BK,
                                              lds + ((kt + NS - 1) % NS) * Cfg::STAGE, wave, lane);
    const char* at = cur;
    const char* bt = cur + Cfg::A_BYTES;
#pragma unroll
    for (int s = 0; s < NKK; ++s) {
      LpFrag<EB> fa[SUB], fb[SUB];
#pragma unroll
      for (int i = 0; i < SUB; ++i) {
        if (TA == 0) lp_frag_kmajor<EB, BK, MB, KSTEP>(fa[i], at, wm0 + MB * i + rb, s, kh);
        else lp_frag_mnmajor<EB, BM>(fa[i], at, wm0 + MB * i + gcol, s * KSTEP + kh, j16);
        if (TB == 1) lp_frag_kmajor<EB, BK, MB, KSTEP>(fb[i], bt, wn0 + MB * i + rb, s, kh);
        else lp_frag_mnmajor<EB, BN>(fb[i], bt, wn0 + MB * i + gcol, s * KSTEP + kh, j16);
      }
#pragma unroll
      for (int i = 0; i < SUB; ++i)
#pragma unroll
        for (int j = 0; j < SUB; ++j) lp_mfma(fa[i], fb[j], acc[i][j]);
    }
  }

  float* __restrict__ Cg = args.C + bz * args.sC;
  const float beta = args.beta;
#pragma unroll
  for (int i = 0; i < SUB; ++i)
#pragma unroll
    for (int j = 0; j < SUB; ++j)
#pragma unroll
      for (int r = 0; r < NACC; ++r) {
        const int br = MB == 16 ? (lane >> 4) * 4 + r : (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        const int64_t gi = m0 + wm0 + MB * i + br;
        const int64_t gj = n0 + wn0 + MB * j + rb;
        if (gi < M && gj < N) {
          float* p = Cg + gi * args.ldc + gj;
          float out = scale * acc[i][j][r];
          if (beta != 0.f) out = fmaf(beta, *p, out);
          *p = out;
        }
      }
}

template <int EB, int BM, int BN, int T, int BK, int TA, int TB>
__global__ void __launch_bounds__(BM * BN / (T * T))
__attribute__((amdgpu_waves_per_eu(LpDmaCfg<EB, BM, BN, T, BK, TA, TB>::OCC, 8)))
gemm_lp_dma_kernel(GemmArgs args) {
  using Cfg = LpDmaCfg<EB, BM, BN, T, BK, TA, TB>;
  __shared__ __attribute__((aligned(16))) char lds[Cfg::LDS_BYTES];
  int tm, tn;
  int64_t bz;
  block_coords(blockIdx.x, args.tiles_m, args.tiles_n, args.batch, tm, tn, bz);
  lp_dma_tile<EB, BM, BN, T, BK, TA, TB>(args, tm, tn, bz, lds);
}

// Operands whose rows all start on 16-byte boundaries take the DMA pipeline,
// any other the register-staged kernel.
template <int EB, int BM, int BN, int T, int BK, int TA, int TB>
hipError_t launch_gemm_lp(const GemmArgs& a, hipStream_t stream) {
  using Cfg = GemmLpCfg<EB, BM, BN, T, BK, TA, TB>;
  if (a.vecA == LP_ALIGN_DMA && a.vecB == LP_ALIGN_DMA)
    return launch_flat<EB>(gemm_lp_dma_kernel<EB, BM, BN, T, BK, TA, TB>, a, BM, BN, Cfg::NT,
                           stream);
  GemmArgs g = a;
  if (g.vecA == LP_ALIGN_DMA) g.vecA = LP_ALIGN_ROWS;
  if (g.vecB == LP_ALIGN_DMA) g.vecB = LP_ALIGN_ROWS;
  return launch_flat<EB>(gemm_lp_kernel<EB, BM, BN, T, BK, TA, TB>, g, BM, BN, Cfg::NT, stream);
}

}  // namespace kt
