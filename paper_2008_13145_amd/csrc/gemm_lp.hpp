// Low-precision GEMM family for gfx950: BF16 or FP8-e4m3 inputs, FP32
// accumulation and output.  C_b = alpha * s * op(A_b) * op(B_b) + beta * C_b
// with s = 1 for BF16 and s = 1 / (scaleA * scaleB) for per-tensor-scaled FP8.
//
// Same configuration knobs as the FP32 family (work-group tile BM x BN, per
// wave an (8T) x (8T) block, K depth BK per LDS stage), with T in
// {2, 4, 8, 16}: T = 2 is one 16x16 MFMA block per wave (16x16x32 BF16,
// 16x16x128 FP8), T = 4 one 32x32 block, T = 8 a 2x2 and T = 16 a 4x4 grid
// of them (the 4x4 grid keeps its 256 accumulators in AGPRs and halves the
// LDS bytes read per MFMA against the 2x2 grid).
// BF16 runs v_mfma_f32_32x32x16_bf16 (8 consecutive K values per lane, lane
// l: row l % 32, K offset 8 * (l / 32)); FP8 runs the 64-deep
// v_mfma_scale_f32_32x32x64_f8f6f4 with unit block scales (32 K bytes per
// lane, K offset 32 * (l / 32)).  A and B fragments take K in the same lane
// order, so each product pairs the right elements whatever order the unit
// sums them in.  Both operands sit in LDS with K contiguous ([m][k], [n][k])
// and every fragment is one (BF16) or two (FP8) 16-byte LDS reads.  Rows are
// padded by 16 bytes so the rows a read phase touches start on different
// banks.  An operand stored contiguous along K is copied into LDS with
// 16-byte vectors; one stored contiguous along M / N is transposed in
// registers, 8 K rows at a time, and written as K-contiguous vectors.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "gemm_f32.hpp"

namespace kt {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4u __attribute__((ext_vector_type(4), aligned(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x8a16 __attribute__((ext_vector_type(8), aligned(16)));

template <int EB>   // element bytes: 2 = BF16, 1 = FP8 e4m3
struct LpElem;
template <>
struct LpElem<2> { typedef uint16_t T; static constexpr int KSTEP = 16, KSTEP16 = 32; };
template <>
struct LpElem<1> { typedef uint8_t T; static constexpr int KSTEP = 64, KSTEP16 = 128; };

// Operand alignment modes (GemmArgs::vecA / vecB for the low-precision
// kernels): 2 = every row starts on a 4-byte boundary; 1 = only the operand's
// base does (odd leading dimension or batch stride); 0 = unaligned base.
enum { LP_ALIGN_NONE = 0, LP_ALIGN_BASE = 1, LP_ALIGN_ROWS = 2 };

// WD dwords from byte address p, which need not be 4-byte aligned: the
// dword-aligned window covering them (one dword more) is read with the widest
// 4-byte-aligned vector loads and realigned with v_alignbyte.  The caller
// guarantees that the window lies inside valid memory (the window never
// starts below a 4-byte aligned base and its extra bytes are columns of the
// same row).
template <int WD>
__device__ __forceinline__ void load_realigned(const void* p, uint32_t* out) {
  static_assert(WD == 1 || WD == 2 || WD == 4, "window of 1, 2 or 4 dwords");
  typedef uint32_t u32x2u __attribute__((ext_vector_type(2), aligned(4)));
  const uintptr_t a = (uintptr_t)p;
  const uint32_t mis = (uint32_t)(a & 3u);
  const uint32_t* w = reinterpret_cast<const uint32_t*>(a - mis);
  uint32_t t[WD + 1];
  if (WD == 4) {
    const u32x4u lo = *reinterpret_cast<const u32x4u*>(w);
    t[0] = lo[0]; t[1] = lo[1]; t[2] = lo[2]; t[3] = lo[3];
    t[WD] = w[4];
  } else if (WD == 2) {
    const u32x2u lo = *reinterpret_cast<const u32x2u*>(w);
    t[0] = lo[0]; t[1] = lo[1];
    t[WD] = w[2];
  } else {
    const u32x2u lo = *reinterpret_cast<const u32x2u*>(w);
    t[0] = lo[0]; t[1] = lo[1];
  }
#pragma unroll
  for (int d = 0; d < WD; ++d) out[d] = __builtin_amdgcn_alignbyte(t[d + 1], t[d], mis);
}

// Global -> register staging of a ROWS x COLS tile (COLS contiguous in memory,
// row stride ld elements), in 16-byte chunks.  Out-of-range elements read 0.
template <int EB, int ROWS, int COLS, int NT>
struct LpTileLoader {
  typedef typename LpElem<EB>::T E;
  static constexpr int EPC = 16 / EB;                 // elements per chunk
  static constexpr int CV = COLS / EPC;               // chunks per row
  static constexpr int NV = ROWS * CV;
  static constexpr int VPT = (NV + NT - 1) / NT;
  static_assert(COLS % EPC == 0, "tile row must hold whole 16-byte chunks");
  u32x4 v[VPT];

  __device__ __forceinline__ void load(const E* __restrict__ base, int64_t ld, int64_t row0,
                                       int64_t col0, int64_t row_lim, int64_t col_lim, int vec,
                                       int tid) {
    const bool rows_in = row0 + ROWS <= row_lim;
    if (vec == LP_ALIGN_ROWS && rows_in && col0 + COLS <= col_lim) {
      // interior tile, rows on 4-byte boundaries: one 16-byte load per chunk
#pragma unroll
      for (int i = 0; i < VPT; ++i) {
        const int c = tid + i * NT;
        if (NV % NT != 0 && c >= NV) { v[i] = u32x4{0u, 0u, 0u, 0u}; continue; }
        const int r = c / CV, q = (c % CV) * EPC;
        v[i] = *reinterpret_cast<const u32x4u*>(base + (row0 + r) * ld + col0 + q);
      }
      return;
    }
    if (vec == LP_ALIGN_BASE && rows_in && col0 + COLS + 4 / EB <= col_lim) {
      // interior tile, rows off 4-byte boundaries: realigned windows, whose
      // extra dword is still inside the row
#pragma unroll
      for (int i = 0; i < VPT; ++i) {
        const int c = tid + i * NT;
        if (NV % NT != 0 && c >= NV) { v[i] = u32x4{0u, 0u, 0u, 0u}; continue; }
        const int r = c / CV, q = (c % CV) * EPC;
        uint32_t o[4];
        load_realigned<4>(base + (row0 + r) * ld + col0 + q, o);
        v[i] = u32x4{o[0], o[1], o[2], o[3]};
      }
      return;
    }
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int c = tid + i * NT;
      if (NV % NT != 0 && c >= NV) { v[i] = u32x4{0u, 0u, 0u, 0u}; continue; }
      const int r = c / CV, q = (c % CV) * EPC;
      const int64_t gr = row0 + r, gc = col0 + q;
      const E* p = base + gr * ld + gc;
      u32x4 t = {0u, 0u, 0u, 0u};
      if (gr < row_lim) {
        if (vec == LP_ALIGN_ROWS && gc + EPC <= col_lim) {
          t = *reinterpret_cast<const u32x4u*>(p);
        } else if (vec == LP_ALIGN_BASE && gc + EPC + 4 / EB <= col_lim) {
          uint32_t o[4];
          load_realigned<4>(p, o);
          t = u32x4{o[0], o[1], o[2], o[3]};
        } else {
          // element by element, packed little-endian into the chunk
#pragma unroll
          for (int e = 0; e < EPC; ++e) {
            const uint32_t x = (gc + e < col_lim) ? (uint32_t)p[e] : 0u;
            t[(e * EB) / 4] |= x << (8 * ((e * EB) % 4));
          }
        }
      }
      v[i] = t;
    }
  }

  // DIRECT: element (r, c) -> lds[r * LD + c] (16-byte stores).
  // TRANSPOSE: element (r, c) -> lds[c * LD + r] (element stores).
  template <bool TRANSPOSE, int LD>
  __device__ __forceinline__ void store(E* lds, int tid) const {
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int c = tid + i * NT;
      if (NV % NT != 0 && c >= NV) continue;
      const int r = c / CV, q = (c % CV) * EPC;
      if (TRANSPOSE) {
#pragma unroll
        for (int e = 0; e < EPC; ++e)
          lds[(q + e) * LD + r] = (E)(v[i][(e * EB) / 4] >> (8 * ((e * EB) % 4)));
      } else {
        *reinterpret_cast<u32x4*>(lds + r * LD + q) = v[i];
      }
    }
  }
};

// Staging of a K x COLS tile whose COLS dimension is contiguous in memory
// (op(A) stored K x M, or op(B) stored K x N), for an LDS layout with K
// contiguous ([col][k]).  Each unit is 8 rows of K by a W-byte chunk of
// columns (W = 4, 8 or 16, sized so the units spread over all threads): the
// 8 chunks are loaded, transposed in registers with byte permutes, and
// written as one 8-deep K run per column (16 bytes for BF16, 8 bytes for
// FP8), in a lane order chosen per unit width (see KFIRST).
template <int EB, int KROWS, int COLS, int NT>
struct LpTransposeLoader {
  typedef typename LpElem<EB>::T E;
  static constexpr int TILE_BYTES = KROWS * COLS * EB;
  static constexpr int W = (TILE_BYTES >= 8 * 16 * NT) ? 16 : (TILE_BYTES >= 8 * 8 * NT) ? 8 : 4;
  static constexpr int WD = W / 4;                    // dwords per row chunk
  static constexpr int EPC = W / EB;                  // columns per unit
  static constexpr int CU = COLS / EPC;               // units across the columns
  static constexpr int KU = KROWS / 8;                // units along K
  static constexpr int NU = KU * CU;                  // units in the tile
  // Lane -> unit order.  Units of 8 or more columns (16-byte chunks for
  // BF16, 8- or 16-byte chunks for FP8) go K-first: neighbouring lanes take
  // neighbouring K units of the same columns, so a store instruction fills
  // consecutive runs of one LDS row, while each global load still covers
  // row segments of 64 bytes or more.  Narrower units go column-first, where
  // coalescing the global loads matters more than the LDS bank spread.
  static constexpr bool KFIRST = EPC >= 8;
  static constexpr int UPT = (NU + NT - 1) / NT;
  static_assert(KROWS % 8 == 0 && COLS % EPC == 0, "tile must hold whole units");
  uint32_t v[UPT][8][WD];

  __device__ __forceinline__ void load(const E* __restrict__ base, int64_t ld, int64_t k0,
                                       int64_t col0, int64_t k_lim, int64_t col_lim, int vec,
                                       int tid) {
    const bool rows_in = k0 + KROWS <= k_lim;
    if (vec == LP_ALIGN_ROWS && rows_in && col0 + COLS <= col_lim) {
      // interior tile, rows on 4-byte boundaries: one straight run of loads
#pragma unroll
      for (int i = 0; i < UPT; ++i) {
        const int u = tid + i * NT;
        if (NU % NT != 0 && u >= NU) continue;
        const int ku = KFIRST ? u % KU : u / CU, cu = KFIRST ? u / KU : u % CU;
        const E* p0 = base + (k0 + ku * 8) * ld + col0 + cu * EPC;
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
          for (int d = 0; d < WD; ++d) v[i][r][d] = reinterpret_cast<const uint32_t*>(p0 + r * ld)[d];
      }
      return;
    }
    if (vec == LP_ALIGN_BASE && rows_in && col0 + COLS + 4 / EB <= col_lim) {
      // interior tile, rows off 4-byte boundaries: realigned windows
#pragma unroll
      for (int i = 0; i < UPT; ++i) {
        const int u = tid + i * NT;
        if (NU % NT != 0 && u >= NU) continue;
        const int ku = KFIRST ? u % KU : u / CU, cu = KFIRST ? u / KU : u % CU;
        const E* p0 = base + (k0 + ku * 8) * ld + col0 + cu * EPC;
#pragma unroll
        for (int r = 0; r < 8; ++r) load_realigned<WD>(p0 + r * ld, v[i][r]);
      }
      return;
    }
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
      const int u = tid + i * NT;
      if (NU % NT != 0 && u >= NU) continue;
      const int ku = KFIRST ? u % KU : u / CU, cu = KFIRST ? u / KU : u % CU;
      const int64_t gc = col0 + cu * EPC;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int64_t gk = k0 + ku * 8 + r;
        const E* p = base + gk * ld + gc;
        const bool in_rows = gk < k_lim;
        if (vec == LP_ALIGN_ROWS && in_rows && gc + EPC <= col_lim) {
#pragma unroll
          for (int d = 0; d < WD; ++d) v[i][r][d] = reinterpret_cast<const uint32_t*>(p)[d];
        } else if (vec == LP_ALIGN_BASE && in_rows && gc + EPC + 4 / EB <= col_lim) {
          load_realigned<WD>(p, v[i][r]);
        } else {
#pragma unroll
          for (int d = 0; d < WD; ++d) v[i][r][d] = 0u;
          if (in_rows) {
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
              const uint32_t x = (gc + e < col_lim) ? (uint32_t)p[e] : 0u;
              v[i][r][(e * EB) / 4] |= x << (8 * ((e * EB) % 4));
            }
          }
        }
      }
    }
  }

  // lds is [COLS][LD] with K contiguous; the tile's K rows start at k = 0.
  template <int LD>
  __device__ __forceinline__ void store(E* lds, int tid) const {
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
      const int u = tid + i * NT;
      if (NU % NT != 0 && u >= NU) continue;
      const int ku = KFIRST ? u % KU : u / CU, cu = KFIRST ? u / KU : u % CU;
#pragma unroll
      for (int c = 0; c < EPC; ++c) {
        const int d = (c * EB) / 4;
        if (EB == 2) {
          // dword j of column c = (row 2j, row 2j + 1) elements c
          const uint32_t sel = (c & 1) ? 0x07060302u : 0x05040100u;
          u32x4 out;
#pragma unroll
          for (int j = 0; j < 4; ++j) out[j] = __builtin_amdgcn_perm(v[i][2 * j + 1][d], v[i][2 * j][d], sel);
          *reinterpret_cast<u32x4*>(lds + (cu * EPC + c) * LD + ku * 8) = out;
        } else {
          // dword h of column c = bytes c of rows 4h .. 4h + 3
          const int sh = 8 * (c & 3);
          uint32_t w[2];
#pragma unroll
          for (int h = 0; h < 2; ++h)
            w[h] = ((v[i][4 * h + 0][d] >> sh) & 0xFFu) | (((v[i][4 * h + 1][d] >> sh) & 0xFFu) << 8) |
                   (((v[i][4 * h + 2][d] >> sh) & 0xFFu) << 16) | (((v[i][4 * h + 3][d] >> sh) & 0xFFu) << 24);
          typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
          *reinterpret_cast<u32x2*>(lds + (cu * EPC + c) * LD + ku * 8) = u32x2{w[0], w[1]};
        }
      }
    }
  }
};

template <int EB, int BM, int BN, int T, int BK, int TA, int TB>
struct GemmLpCfg {
  static constexpr int WT = 8 * T;
  // T = 2 runs the 16x16 MFMAs (16x16x32 BF16, 16x16x128 FP8), larger T the
  // 32x32 ones (32x32x16 BF16, 32x32x64 FP8).
  static constexpr int MB = T == 2 ? 16 : 32;        // MFMA block edge
  static constexpr int SUB = WT / MB;                // MFMA blocks per wave edge
  static constexpr int KSTEP = T == 2 ? LpElem<EB>::KSTEP16 : LpElem<EB>::KSTEP;
  static constexpr int WAVES_N = BN / WT;
  static constexpr int WAVES = (BM / WT) * WAVES_N;
  static constexpr int NT = WAVES * 64;
  static constexpr int PADK = 16 / EB;               // 16-byte row pad
  static constexpr int LDK = BK + PADK;              // LDS row length (elements)
  static constexpr int A_STAGE = BM * LDK;           // elements
  static constexpr int B_STAGE = BN * LDK;
  static constexpr int LDS_BYTES = 2 * (A_STAGE + B_STAGE) * EB;
  static_assert(T == 2 || T == 4 || T == 8 || T == 16, "low-precision wave blocks of 16 to 128");
  static_assert(BM % WT == 0 && BN % WT == 0, "tile must hold whole wave blocks");
  static_assert(WAVES >= 1 && WAVES <= 16, "1..16 waves per work-group");
  static_assert(BK % KSTEP == 0, "BK multiple of the MFMA depth");
  static_assert(LDS_BYTES <= 160 * 1024, "LDS budget");
};

// One lane's operand fragment for one MFMA: 8 BF16 values (16 bytes) or
// 32 FP8 codes (32 bytes), read from LDS as one or two 16-byte reads.
template <int EB>
struct LpFrag;
template <>
struct LpFrag<2> {
  bf16x8 v;
  __device__ __forceinline__ void read(const void* p) { v = *reinterpret_cast<const bf16x8*>(p); }
};
template <>
struct LpFrag<1> {
  i32x8 v;
  __device__ __forceinline__ void read(const void* p) { v = *reinterpret_cast<const i32x8a16*>(p); }
};

__device__ __forceinline__ void lp_mfma(const LpFrag<2>& a, const LpFrag<2>& b, f32x16& c) {
  c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v, b.v, c, 0, 0, 0);
}

// Operand formats 0 / 0 = e4m3 for A and B; block scales 127 = 2^0 (E8M0).
__device__ __forceinline__ void lp_mfma(const LpFrag<1>& a, const LpFrag<1>& b, f32x16& c) {
  c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a.v, b.v, c, 0, 0, 0, 127, 0, 127);
}

__device__ __forceinline__ void lp_mfma(const LpFrag<2>& a, const LpFrag<2>& b, f32x4& c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, c, 0, 0, 0);
}

__device__ __forceinline__ void lp_mfma(const LpFrag<1>& a, const LpFrag<1>& b, f32x4& c) {
  c = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a.v, b.v, c, 0, 0, 0, 127, 0, 127);
}

// One BM x BN output tile (tile row tm, tile column tn) of batch item bz:
// the whole K loop and the epilogue.  lds holds the two stages of both
// operands; the caller synchronizes before reusing it for another tile.
template <int EB, int BM, int BN, int T, int BK, int TA, int TB>
__device__ __forceinline__ void lp_tile(const GemmArgs& args, int tm, int tn, int64_t bz,
                                        typename LpElem<EB>::T* lds) {
  using Cfg = GemmLpCfg<EB, BM, BN, T, BK, TA, TB>;
  typedef typename LpElem<EB>::T E;
  constexpr int NT = Cfg::NT;
  constexpr int WT = Cfg::WT;
  constexpr int LDK = Cfg::LDK;
  constexpr int MB = Cfg::MB;                // MFMA block edge (16 or 32)
  constexpr int SUB = Cfg::SUB;              // MFMA blocks per wave edge
  E* As = lds;                               // [2][BM][LDK]
  E* Bs = lds + 2 * Cfg::A_STAGE;            // [2][BN][LDK]

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave / Cfg::WAVES_N) * WT;
  const int wn0 = (wave % Cfg::WAVES_N) * WT;

  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int64_t M = args.M, N = args.N, K = args.K;
  const E* __restrict__ Ag = static_cast<const E*>(args.A) + bz * args.sA;
  const E* __restrict__ Bg = static_cast<const E*>(args.B) + bz * args.sB;
  const int vecA = args.vecA, vecB = args.vecB;
  // FP8 per-tensor scales: loaded before the K loop so their latency is hidden
  float scale = args.alpha;
  if (EB == 1) scale = args.alpha / (args.scaleA[0] * args.scaleB[0]);

  // A: TA == 0 -> k contiguous (direct 16-byte copy), TA == 1 -> m contiguous
  // (register transpose).  B: TB == 1 -> direct, TB == 0 -> transpose.
  typedef typename std::conditional<TA == 0, LpTileLoader<EB, BM, BK, NT>,
                                    LpTransposeLoader<EB, BK, BM, NT>>::type LoaderA;
  typedef typename std::conditional<TB == 1, LpTileLoader<EB, BN, BK, NT>,
                                    LpTransposeLoader<EB, BK, BN, NT>>::type LoaderB;
  LoaderA la;
  LoaderB lb;

  auto load_stage = [&](int64_t k0) {
    if (TA) la.load(Ag, args.lda, k0, m0, K, M, vecA, tid);
    else    la.load(Ag, args.lda, m0, k0, M, K, vecA, tid);
    if (TB) lb.load(Bg, args.ldb, n0, k0, N, K, vecB, tid);
    else    lb.load(Bg, args.ldb, k0, n0, K, N, vecB, tid);
  };
  auto store_stage = [&](int buf) {
    if constexpr (TA == 0) la.template store<false, LDK>(As + buf * Cfg::A_STAGE, tid);
    else                   la.template store<LDK>(As + buf * Cfg::A_STAGE, tid);
    if constexpr (TB == 1) lb.template store<false, LDK>(Bs + buf * Cfg::B_STAGE, tid);
    else                   lb.template store<LDK>(Bs + buf * Cfg::B_STAGE, tid);
  };

  typedef typename std::conditional<MB == 16, f32x4, f32x16>::type Acc;
  constexpr int NACC = MB == 16 ? 4 : 16;
  Acc acc[SUB][SUB];
#pragma unroll
  for (int i = 0; i < SUB; ++i)
#pragma unroll
    for (int j = 0; j < SUB; ++j)
#pragma unroll
      for (int r = 0; r < NACC; ++r) acc[i][j][r] = 0.f;

  // lane l feeds row l % MB of its block with K values from group l / MB
  constexpr int KSTEP = Cfg::KSTEP;
  const int rb = lane % MB, kh = (lane / MB) * (KSTEP * MB / 64);
  const int nk = (int)((K + BK - 1) / BK);
  if (nk > 0) {
    load_stage(0);
    store_stage(0);
    __syncthreads();
  }
  constexpr int NKK = BK / KSTEP;
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    const E* as = As + buf * Cfg::A_STAGE;
    const E* bs = Bs + buf * Cfg::B_STAGE;
    if (kt + 1 < nk) load_stage((int64_t)(kt + 1) * BK);
#pragma unroll
    for (int s = 0; s < NKK; ++s) {
      LpFrag<EB> fa[SUB], fb[SUB];
#pragma unroll
      for (int i = 0; i < SUB; ++i) {
        fa[i].read(as + (wm0 + MB * i + rb) * LDK + s * KSTEP + kh);
        fb[i].read(bs + (wn0 + MB * i + rb) * LDK + s * KSTEP + kh);
      }
#pragma unroll
      for (int i = 0; i < SUB; ++i)
#pragma unroll
        for (int j = 0; j < SUB; ++j) lp_mfma(fa[i], fb[j], acc[i][j]);
    }
    if (kt + 1 < nk) store_stage(buf ^ 1);
    __syncthreads();
  }

  float* __restrict__ Cg = args.C + bz * args.sC;
  const float beta = args.beta;
#pragma unroll
  for (int i = 0; i < SUB; ++i)
#pragma unroll
    for (int j = 0; j < SUB; ++j)
#pragma unroll
      for (int r = 0; r < NACC; ++r) {
        // 32x32 blocks: row (r / 4) * 8 + (lane / 32) * 4 + r % 4; 16x16
        // blocks: row (lane / 16) * 4 + r; the column is lane % MB
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
gemm_lp_kernel(GemmArgs args) {
  using Cfg = GemmLpCfg<EB, BM, BN, T, BK, TA, TB>;
  typedef typename LpElem<EB>::T E;
  __shared__ __attribute__((aligned(16))) E lds[Cfg::LDS_BYTES / EB];
  int tm, tn;
  int64_t bz;
  block_coords(blockIdx.x, args.tiles_m, args.tiles_n, args.batch, tm, tn, bz);
  lp_tile<EB, BM, BN, T, BK, TA, TB>(args, tm, tn, bz, lds);
}

}  // namespace kt
