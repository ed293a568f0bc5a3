// LDS-DMA pipeline of the FP32 family (T = 2, 4, 8), taken when every
// operand row starts on a 16-byte boundary and no 16-byte read leaves an
// operand (the same rule as the low-precision family, with 4-float chunks).
// Same configuration knobs and results contract as gemm_f32.hpp; the
// differences:
//
// * Tiles move HBM -> LDS by global_load_lds_dwordx4 (1 KiB per wave
//   instruction), NS = 2..4 stages in flight, waited for with vmcnt; no
//   register staging and no LDS stores by the waves.
// * Each operand keeps its stored layout in LDS: K-contiguous operands as
//   [row][k] with 16-byte chunks XOR-swizzled by row (as the low-precision
//   tiles), M/N-contiguous ones as [k][col].
// * The MFMA's K positions are assigned by lane group instead of
//   interleaved: for the 32x32x2 MFMA lane half h takes k = h * BK / 2 + q at
//   step q, for the 16x16x4 MFMA lane quarter g takes k = g * BK / 4 + q, so a
//   lane reads consecutive k of one row of a K-contiguous tile.  A and B use
//   the same assignment, so each product pairs matching elements; the sums
//   run in another order than the register-staged kernel's (same bound).
#pragma once
#include "gemm_lp_dma.hpp"

namespace kt {

template <int BM, int BN, int T, int BK, int TA, int TB>
struct F32DmaCfg {
  using Base = GemmF32Cfg<BM, BN, T, BK, TA, TB>;
  static constexpr int NT = Base::NT, WAVES = Base::WAVES, WT = Base::WT;
  static constexpr int A_BYTES = BM * BK * 4, B_BYTES = BN * BK * 4;
  static constexpr int STAGE = A_BYTES + B_BYTES;
  static constexpr int BUDGET = 64 * 1024;
  static constexpr int NS_FIT = BUDGET / STAGE;
  static constexpr int NS = NS_FIT < 2 ? 2 : (NS_FIT > 4 ? 4 : NS_FIT);
  static constexpr int LDS_BYTES = NS * STAGE;
  static constexpr int NBA = A_BYTES / 1024, NBB = B_BYTES / 1024;
  static constexpr int NBLK = NBA + NBB;
  static constexpr int NW_LO = NBLK / WAVES, NW_HI = (NBLK + WAVES - 1) / WAVES;
  // a K-major row is BK floats: 2..16 chunks of 16 bytes
  static constexpr int KCPR = BK / 4;
  static_assert(T >= 2, "the 4x4x1 family keeps the register-staged pipeline");
  static_assert(A_BYTES % 1024 == 0 && B_BYTES % 1024 == 0, "tiles of whole 1 KiB blocks");
  static_assert(LDS_BYTES <= 160 * 1024, "LDS budget");
  static_assert((NS - 2) * NW_HI < 64, "vmcnt range");
  // An M/N-contiguous row must be whole chunks; a 1 KiB block must hold whole rows.
  static_assert((BM * 4) % 16 == 0 && (BN * 4) % 16 == 0, "whole chunks per row");
};

// M/N-major FP32 rows (one k each, COLS floats = CPR 16-byte chunks): the
// lane groups of an MFMA step read the same columns of rows BK/2 apart
// (32x32x2: two halves of 32 lanes, 128 bytes each) or BK/4 apart (16x16x4:
// four quarters of 16 lanes, 64 bytes each), which would fall on the same
// banks of a 256-byte bank line; XOR-ing a group's chunk index by 8 (halves)
// or by 4 x its quarter (quarters) puts the groups on different banks.
template <int CPR, int BK, int T>
__device__ __forceinline__ int f32_mswz(int k) {
  if constexpr (T == 2) return CPR >= 8 ? (((k / (BK / 4)) & 3) * 4) % CPR : 0;
  else return CPR >= 16 ? ((k / (BK / 2)) & 1) * 8 : 0;
}

template <int BM, int BN, int T, int BK, int TA, int TB>
__device__ __forceinline__ void f32_dma_issue(const GemmArgs& args, const char* __restrict__ Ag,
                                              const char* __restrict__ Bg, int64_t m0, int64_t n0,
                                              int64_t k0, char* stage, int wave, int lane) {
  using Cfg = F32DmaCfg<BM, BN, T, BK, TA, TB>;
  constexpr int CE = 4;
#pragma unroll
  for (int i = 0; i < Cfg::NW_HI; ++i) {
    const int q = wave + i * Cfg::WAVES;
    if (q >= Cfg::NBLK) break;   // wave-uniform
    const bool isA = q < Cfg::NBA;
    const int blk = isA ? q : q - Cfg::NBA;
    const int o = blk * 1024 + lane * 16;
    const bool kmajor = isA ? (TA == 0) : (TB == 1);
    const int cols = isA ? BM : BN;
    const int64_t lim = isA ? args.M : args.N;
    const int64_t ld = isA ? args.lda : args.ldb;
    const int64_t c0 = isA ? m0 : n0;
    const char* base = isA ? Ag : Bg;
    int64_t elem;
    if (kmajor) {
      constexpr int ROWB = BK * 4;
      const int r = o / ROWB, p = (o % ROWB) / 16;
      const int c = p ^ kswz<Cfg::KCPR>(r);
      int64_t row = c0 + r;
      row = row < lim ? row : lim - 1;
      int64_t kk = k0 + (int64_t)c * CE;
      kk = kk < args.K ? kk : ((args.K - 1) / CE) * CE;
      elem = row * ld + kk;
    } else {
      const int ROWB = cols * 4, CPR = ROWB / 16;
      const int k = o / ROWB, p = (o % ROWB) / 16;
      int c;
      if (isA) c = p ^ f32_mswz<BM / 4, BK, T>(k);
      else c = p ^ f32_mswz<BN / 4, BK, T>(k);
      int64_t kr = k0 + k;
      kr = kr < args.K ? kr : args.K - 1;
      int64_t col = c0 + (int64_t)c * CE;
      col = col < lim ? col : ((lim - 1) / CE) * CE;
      elem = kr * ld + col;
    }
    char* dst = stage + (isA ? 0 : Cfg::A_BYTES) + blk * 1024;
    __builtin_amdgcn_global_load_lds((gbl_void_t*)(base + elem * 4), (lds_void_t*)dst, 16, 0, 0);
  }
}

template <int BM, int BN, int T, int BK, int TA, int TB>
__device__ __forceinline__ void f32_dma_zero_tail(char* stage, int kvalid, int tid) {
  using Cfg = F32DmaCfg<BM, BN, T, BK, TA, TB>;
#pragma unroll
  for (int op = 0; op < 2; ++op) {
    const bool kmajor = op == 0 ? (TA == 0) : (TB == 1);
    const int cols = op == 0 ? BM : BN;
    float* t = reinterpret_cast<float*>(stage + (op == 0 ? 0 : Cfg::A_BYTES));
    const int tail = BK - kvalid;
    if (kmajor) {
      for (int i = tid; i < cols * tail; i += Cfg::NT) {
        const int r = i / tail, k = kvalid + i % tail;
        t[r * BK + ((k >> 2) ^ kswz<Cfg::KCPR>(r)) * 4 + (k & 3)] = 0.f;
      }
    } else {
      for (int i = tid; i < cols * tail; i += Cfg::NT) t[kvalid * cols + i] = 0.f;
    }
  }
}

// Element (row, k) of a K-major tile / (k, col) of an M/N-major tile.
template <int BK>
__device__ __forceinline__ float f32_at_kmajor(const float* t, int row, int k) {
  return t[row * BK + ((k >> 2) ^ kswz<BK / 4>(row)) * 4 + (k & 3)];
}
template <int COLS, int BK, int T>
__device__ __forceinline__ float f32_at_mnmajor(const float* t, int k, int col) {
  constexpr int CPR = COLS / 4;
  return t[k * COLS + (((col >> 2) ^ f32_mswz<CPR, BK, T>(k)) << 2) + (col & 3)];
}

template <int BM, int BN, int T, int BK, int TA, int TB>
__global__ void __launch_bounds__(BM * BN / (T * T))
gemm_f32_dma_kernel(GemmArgs args) {
  using Cfg = F32DmaCfg<BM, BN, T, BK, TA, TB>;
  constexpr int NS = Cfg::NS;
  constexpr int WT = Cfg::WT;
  __shared__ __attribute__((aligned(16))) char lds[Cfg::LDS_BYTES];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave / Cfg::Base::WAVES_N) * WT;
  const int wn0 = (wave % Cfg::Base::WAVES_N) * WT;
  int tm, tn;
  int64_t bz;
  block_coords(blockIdx.x, args.tiles_m, args.tiles_n, args.batch, tm, tn, bz);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int64_t M = args.M, N = args.N, K = args.K;
  const char* __restrict__ Ag = static_cast<const char*>(args.A) + bz * args.sA * 4;
  const char* __restrict__ Bg = static_cast<const char*>(args.B) + bz * args.sB * 4;

  auto A_at = [&](const float* t, int m, int k) {
    if constexpr (TA == 0) return f32_at_kmajor<BK>(t, m, k);
    else return f32_at_mnmajor<BM, BK, T>(t, k, m);
  };
  auto B_at = [&](const float* t, int n, int k) {
    if constexpr (TB == 1) return f32_at_kmajor<BK>(t, n, k);
    else return f32_at_mnmajor<BN, BK, T>(t, k, n);
  };
  // Four consecutive k (k0 a multiple of 4) of one row / column: one 16-byte
  // LDS read from a K-major tile (a whole swizzled chunk), four from an
  // M/N-major one.
  auto A4 = [&](const float* t, int m, int k0) {
    if constexpr (TA == 0)
      return *reinterpret_cast<const f32x4*>(t + m * BK + ((k0 >> 2) ^ kswz<BK / 4>(m)) * 4);
    else
      return f32x4{A_at(t, m, k0), A_at(t, m, k0 + 1), A_at(t, m, k0 + 2), A_at(t, m, k0 + 3)};
  };
  auto B4 = [&](const float* t, int n, int k0) {
    if constexpr (TB == 1)
      return *reinterpret_cast<const f32x4*>(t + n * BK + ((k0 >> 2) ^ kswz<BK / 4>(n)) * 4);
    else
      return f32x4{B_at(t, n, k0), B_at(t, n, k0 + 1), B_at(t, n, k0 + 2), B_at(t, n, k0 + 3)};
  };

  constexpr int NACC = (T == 2) ? 4 : (T == 4) ? 16 : 64;
  float acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = 0.f;

  const int nk = (int)((K + BK - 1) / BK);
  const int my_blocks = (wave < Cfg::NBLK % Cfg::WAVES || Cfg::NBLK % Cfg::WAVES == 0)
                            ? Cfg::NW_HI : Cfg::NW_LO;
#pragma unroll
  for (int s = 0; s < NS - 1; ++s)
    if (s < nk)
      f32_dma_issue<BM, BN, T, BK, TA, TB>(args, Ag, Bg, m0, n0, (int64_t)s * BK,
                                           lds + s * Cfg::STAGE, wave, lane);

  for (int kt = 0; kt < nk; ++kt) {
    const int ahead = min(NS - 2, nk - 1 - kt);
    if (my_blocks == Cfg::NW_HI) wait_stage<Cfg::NW_HI, NS>(ahead);
    else wait_stage<Cfg::NW_LO, NS>(ahead);
    char* cur = lds + (kt % NS) * Cfg::STAGE;
    if (kt == nk - 1 && K - (int64_t)kt * BK < BK) {
      f32_dma_zero_tail<BM, BN, T, BK, TA, TB>(cur, (int)(K - (int64_t)kt * BK), tid);
      vm_wait_barrier<0>();
    }
    if (kt + NS - 1 < nk)
      f32_dma_issue<BM, BN, T, BK, TA, TB>(args, Ag, Bg, m0, n0, (int64_t)(kt + NS - 1) * BK,
                                           lds + ((kt + NS - 1) % NS) * Cfg::STAGE, wave, lane);
    const float* as = reinterpret_cast<const float*>(cur);
    const float* bs = reinterpret_cast<const float*>(cur + Cfg::A_BYTES);
    if constexpr (T == 2) {
      // 16x16x4: lane quarter g = lane / 16 takes k = g * BK / 4 + q
      const int r16 = lane & 15, g = lane >> 4;
      constexpr int KQ = BK / 4;
      f32x4 c = {acc[0], acc[1], acc[2], acc[3]};
      // element reads, which the compiler merges where it can (explicit
      // 16-byte reads measured 3 % slower here on the mixed layouts)
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        const float a = A_at(as, wm0 + r16, g * KQ + q);
        const float b = B_at(bs, wn0 + r16, g * KQ + q);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = c[r];
    } else if constexpr (T == 4) {
      const int r32 = lane & 31, h = lane >> 5;
      constexpr int KH = BK / 2;
      f32x16 c;
#pragma unroll
      for (int r = 0; r < 16; ++r) c[r] = acc[r];
      static_assert(KH % 4 == 0, "whole 16-byte chunks per lane half");
#pragma unroll
      for (int q0 = 0; q0 < KH; q0 += 4) {
        const f32x4 a = A4(as, wm0 + r32, h * KH + q0);
        const f32x4 b = B4(bs, wn0 + r32, h * KH + q0);
#pragma unroll
        for (int u = 0; u < 4; ++u) c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[u], b[u], c, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = c[r];
    } else {
      const int r32 = lane & 31, h = lane >> 5;
      constexpr int KH = BK / 2;
      f32x16 c00, c01, c10, c11;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        c00[r] = acc[r]; c01[r] = acc[16 + r]; c10[r] = acc[32 + r]; c11[r] = acc[48 + r];
      }
      static_assert(KH % 4 == 0, "whole 16-byte chunks per lane half");
#pragma unroll
      for (int q0 = 0; q0 < KH; q0 += 4) {
        const int k = h * KH + q0;
        const f32x4 a0 = A4(as, wm0 + r32, k), a1 = A4(as, wm0 + 32 + r32, k);
        const f32x4 b0 = B4(bs, wn0 + r32, k), b1 = B4(bs, wn0 + 32 + r32, k);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          c00 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[u], b0[u], c00, 0, 0, 0);
          c01 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[u], b1[u], c01, 0, 0, 0);
          c10 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[u], b0[u], c10, 0, 0, 0);
          c11 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[u], b1[u], c11, 0, 0, 0);
        }
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        acc[r] = c00[r]; acc[16 + r] = c01[r]; acc[32 + r] = c10[r]; acc[48 + r] = c11[r];
      }
    }
  }

  float* __restrict__ Cg = args.C + bz * args.sC;
  const float alpha = args.alpha, beta = args.beta;
  const int64_t ldc = args.ldc;
  auto put = [&](int row, int col, float v) {
    const int64_t gi = m0 + wm0 + row, gj = n0 + wn0 + col;
    if (gi < M && gj < N) {
      float* p = Cg + gi * ldc + gj;
      float out = alpha * v;
      if (beta != 0.f) out = fmaf(beta, *p, out);
      *p = out;
    }
  };
  if constexpr (T == 2) {
#pragma unroll
    for (int r = 0; r < 4; ++r) put((lane >> 4) * 4 + r, lane & 15, acc[r]);
  } else if constexpr (T == 4) {
#pragma unroll
    for (int r = 0; r < 16; ++r) put((r >> 2) * 8 + (lane >> 5) * 4 + (r & 3), lane & 31, acc[r]);
  } else {
#pragma unroll
    for (int sub = 0; sub < 4; ++sub) {
      const int si = sub >> 1, sj = sub & 1;
#pragma unroll
      for (int r = 0; r < 16; ++r)
        put(32 * si + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3), 32 * sj + (lane & 31),
            acc[16 * (2 * si + sj) + r]);
    }
  }
}

// Configurations the DMA pipeline serves: the 16x16 and 32x32 MFMA families
// whose tiles are whole 1 KiB DMA blocks.
template <int BM, int BN, int T, int BK>
struct F32DmaServes {
  static constexpr bool value = T >= 2 && (BM * BK * 4) % 1024 == 0 && (BN * BK * 4) % 1024 == 0;
};

// Host-side launcher of one instantiation on a stream: operands whose rows
// all start on 16-byte boundaries take the DMA pipeline where the
// configuration has one, any other the register-staged kernel.
template <int BM, int BN, int T, int BK, int TA, int TB>
hipError_t launch_gemm_f32(const GemmArgs& a, hipStream_t stream) {
  using Cfg = GemmF32Cfg<BM, BN, T, BK, TA, TB>;
  if constexpr (F32DmaServes<BM, BN, T, BK>::value) {
    if (a.vecA == LP_ALIGN_DMA && a.vecB == LP_ALIGN_DMA)
      return launch_flat<4>(gemm_f32_dma_kernel<BM, BN, T, BK, TA, TB>, a, BM, BN, Cfg::NT, stream);
  }
  return launch_flat<4>(gemm_f32_kernel<BM, BN, T, BK, TA, TB>, a, BM, BN, Cfg::NT, stream);
}

}  // namespace kt
