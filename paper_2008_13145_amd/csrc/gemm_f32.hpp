// FP32 tiled GEMM family for gfx950: C_b = alpha * op(A_b) * op(B_b) + beta * C_b.
//
// One kernel template covers the whole configuration space.  The paper's
// kernel (section 3) gives each work item an R x A tile of the left input and
// an A x C tile of the right one, with no local memory; on CDNA4 the same
// three knobs become: a BM x BN work-group tile staged through LDS in BK-deep
// slices (double buffered), and a per-wave (8T) x (8T) output block computed
// by MFMA, i.e. T*T accumulators per lane:
//
//   T = 1: 8x8 wave block, v_mfma_f32_4x4x1f32 (16 blocks): 4 output blocks
//          x 4-way K split, reduced with cross-lane shuffles at the end;
//   T = 2: 16x16 wave block, v_mfma_f32_16x16x4f32;
//   T = 4: 32x32 wave block, v_mfma_f32_32x32x2f32;
//   T = 8: 64x64 wave block, 2x2 v_mfma_f32_32x32x2f32.
//
// LDS holds both operands K-major (As[k][m], Bs[k][n]) so every MFMA operand
// read is a run of consecutive addresses.  An operand whose global storage
// is contiguous along K is transposed on the way in (row pad 2 keeps those
// scattered writes on distinct banks); an operand contiguous along M/N is
// copied straight (no pad, 16-byte vector writes).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kt {

struct GemmArgs {
  int64_t M, N, K, batch;
  const void* A; int64_t lda, sA;
  const void* B; int64_t ldb, sB;
  float* C; int64_t ldc, sC;
  float alpha, beta;
  const float* scaleA; const float* scaleB;   // FP8 only
  int32_t vecA, vecB;   // low-precision paths: row alignment mode (LP_ALIGN_*)
  int32_t tiles_m, tiles_n;
};

typedef float f32x4 __attribute__((ext_vector_type(4)));
// Four floats with only 4-byte alignment: global_load_dwordx4 needs dword
// alignment on CDNA, so rows of any leading dimension load as 16-byte vectors.
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Work-group id -> (batch item, tile_m, tile_n).  The grid is one flat range
// over (batch item, tile).  Consecutive work-group ids land on different XCDs
// (round robin over 8), so the id is first remapped to give each XCD a
// contiguous range of that flat space -- whole batch items, or neighbouring
// tiles of one item; tiles of an item are then walked in groups of 8
// tile-rows so that neighbours share A row panels and B column panels in that
// XCD's L2.
__device__ __forceinline__ void block_coords(int64_t pid, int tiles_m, int tiles_n,
                                             int64_t batch, int& tm, int& tn, int64_t& bz) {
  const int64_t nt = (int64_t)tiles_m * tiles_n;
  const int64_t per = nt * batch / 8;
  int64_t t = pid;
  if (pid < per * 8) t = (pid % 8) * per + pid / 8;
  bz = t / nt;
  t -= bz * nt;
  const int64_t group = 8;
  const int64_t width = group * tiles_n;
  const int64_t gid = t / width;
  const int64_t first_m = gid * group;
  const int64_t gsz = (tiles_m - first_m) < group ? (tiles_m - first_m) : group;
  const int64_t r = t % width;
  tm = (int)(first_m + r % gsz);
  tn = (int)(r / gsz);
}

// Launches a GEMM family kernel over a flat (batch item, tile) grid, in as
// many launches as the 32-bit work-item count of one grid dimension needs.
// EB is the element size of A and B in bytes.
template <int EB, typename Kernel>
hipError_t launch_flat(Kernel kernel, const GemmArgs& a, int bm, int bn, int nt_threads,
                       hipStream_t stream) {
  GemmArgs g = a;
  g.tiles_m = (int)((a.M + bm - 1) / bm);
  g.tiles_n = (int)((a.N + bn - 1) / bn);
  const int64_t nt = (int64_t)g.tiles_m * g.tiles_n;
  const int64_t max_blocks = (int64_t)0xFFFFFFFFu / nt_threads;
  if (nt > max_blocks) return hipErrorInvalidConfiguration;
  const int64_t per_launch = max_blocks / nt;
  for (int64_t b0 = 0; b0 < a.batch; b0 += per_launch) {
    const int64_t nb = (a.batch - b0) < per_launch ? (a.batch - b0) : per_launch;
    g.batch = nb;
    g.A = static_cast<const char*>(a.A) + b0 * a.sA * EB;
    g.B = static_cast<const char*>(a.B) + b0 * a.sB * EB;
    g.C = a.C + b0 * a.sC;
    hipLaunchKernelGGL(kernel, dim3((unsigned)(nt * nb)), dim3(nt_threads), 0, stream, g);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Global -> register staging of one ROWS x COLS tile whose COLS dimension is
// contiguous in memory (row stride ld).  Rows beyond row_lim or columns beyond
// col_lim read as zero.
template <int ROWS, int COLS, int NT>
struct TileLoader {
  static constexpr int CV = COLS / 4;                 // float4 chunks per row
  static constexpr int NV = ROWS * CV;                // chunks in the tile
  static constexpr int VPT = (NV + NT - 1) / NT;      // chunks per thread
  f32x4 v[VPT];

  __device__ __forceinline__ void load(const float* __restrict__ base, int64_t ld, int64_t row0,
                                       int64_t col0, int64_t row_lim, int64_t col_lim, int tid) {
    const bool full = (row0 + ROWS <= row_lim) && (col0 + COLS <= col_lim);
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int c = tid + i * NT;
      if (NV % NT != 0 && c >= NV) { v[i] = f32x4{0.f, 0.f, 0.f, 0.f}; continue; }
      const int r = c / CV, q = (c % CV) * 4;
      const int64_t gr = row0 + r, gc = col0 + q;
      const float* p = base + gr * ld + gc;
      if (full) {
        v[i] = *reinterpret_cast<const f32x4u*>(p);
      } else {
        f32x4 t = {0.f, 0.f, 0.f, 0.f};
        if (gr < row_lim) {
          if (gc + 4 <= col_lim) {
            t = *reinterpret_cast<const f32x4u*>(p);
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (gc + e < col_lim) t[e] = p[e];
          }
        }
        v[i] = t;
      }
    }
  }

  // Store into an LDS array laid out [COLS][LD] (transpose: element (r, c) goes
  // to lds[c * LD + r]) or [ROWS][LD] (direct: lds[r * LD + c]).
  template <bool TRANSPOSE, int LD>
  __device__ __forceinline__ void store(float* lds, int tid) const {
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int c = tid + i * NT;
      if (NV % NT != 0 && c >= NV) continue;
      const int r = c / CV, q = (c % CV) * 4;
      if (TRANSPOSE) {
#pragma unroll
        for (int e = 0; e < 4; ++e) lds[(q + e) * LD + r] = v[i][e];
      } else {
        *reinterpret_cast<f32x4*>(lds + r * LD + q) = v[i];
      }
    }
  }
};

template <int BM, int BN, int T, int BK, int TA, int TB>
struct GemmF32Cfg {
  static constexpr int WT = 8 * T;                     // wave block edge
  static constexpr int WAVES_M = BM / WT;
  static constexpr int WAVES_N = BN / WT;
  static constexpr int WAVES = WAVES_M * WAVES_N;
  static constexpr int NT = WAVES * 64;
  // A operand tile: op(A) rows m, depth k.  TA == 0 -> stored with k contiguous
  // (transpose into LDS), TA == 1 -> m contiguous (direct copy).
  static constexpr int LDA_S = BM + (TA == 0 ? 2 : 0);
  static constexpr int LDB_S = BN + (TB == 1 ? 2 : 0);
  static constexpr int A_STAGE = BK * LDA_S;
  static constexpr int B_STAGE = BK * LDB_S;
  static constexpr int LDS_FLOATS = 2 * (A_STAGE + B_STAGE);
  // Occupancy target (waves per SIMD): what the LDS footprint allows (160 KiB
  // per CU, 4 SIMDs), capped by an estimate of the registers a wave needs
  // (accumulators, one stage of MFMA operands, the prefetched stage and a
  // fixed allowance for addresses), so the register budget it implies does
  // not force spills.  It lets the T = 8 kernels trade AGPRs for occupancy.
  static constexpr int WG_PER_CU = (160 * 1024) / (LDS_FLOATS * 4) < 16 ? (160 * 1024) / (LDS_FLOATS * 4) : 16;
  static constexpr int OCC_LDS = (WG_PER_CU * WAVES) / 4;
  static constexpr int ACC_REGS = T == 1 ? 4 : T * T;
  static constexpr int OPS_REGS = T <= 2 ? 2 * (BK / 4) : T == 4 ? BK : 4 * (BK / 2 > 16 ? 16 : BK / 2);
  static constexpr int PREF_REGS = 4 * ((BM * BK / 4 + NT - 1) / NT + (BN * BK / 4 + NT - 1) / NT);
  static constexpr int OCC_REG = 512 / (ACC_REGS + OPS_REGS + PREF_REGS + 40);
  static constexpr int OCC_MIN = OCC_LDS < OCC_REG ? OCC_LDS : OCC_REG;
  static constexpr int OCC = OCC_MIN < 1 ? 1 : OCC_MIN > 8 ? 8 : OCC_MIN;
  static_assert(BM % WT == 0 && BN % WT == 0, "tile must hold whole wave blocks");
  static_assert(WAVES >= 1 && WAVES <= 16, "1..16 waves per work-group");
  static_assert(LDS_FLOATS * 4 <= 160 * 1024, "LDS budget");
  static_assert(BK % 4 == 0, "BK multiple of 4");
};

template <int BM, int BN, int T, int BK, int TA, int TB>
__global__ void __launch_bounds__(BM * BN / (T * T))
__attribute__((amdgpu_waves_per_eu(GemmF32Cfg<BM, BN, T, BK, TA, TB>::OCC, 8)))
gemm_f32_kernel(GemmArgs args) {
  using Cfg = GemmF32Cfg<BM, BN, T, BK, TA, TB>;
  constexpr int NT = Cfg::NT;
  constexpr int WT = Cfg::WT;
  __shared__ float lds[Cfg::LDS_FLOATS];
  float* As = lds;                          // [2][BK][LDA_S]
  float* Bs = lds + 2 * Cfg::A_STAGE;       // [2][BK][LDB_S]

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave / Cfg::WAVES_N) * WT;
  const int wn0 = (wave % Cfg::WAVES_N) * WT;

  int tm, tn;
  int64_t bz;
  block_coords(blockIdx.x, args.tiles_m, args.tiles_n, args.batch, tm, tn, bz);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int64_t M = args.M, N = args.N, K = args.K;
  const float* __restrict__ Ag = static_cast<const float*>(args.A) + bz * args.sA;
  const float* __restrict__ Bg = static_cast<const float*>(args.B) + bz * args.sB;

  // Loaders: the tile's contiguous dimension is the loader's COLS.
  TileLoader<(TA ? BK : BM), (TA ? BM : BK), NT> la;
  TileLoader<(TB ? BN : BK), (TB ? BK : BN), NT> lb;

  auto load_stage = [&](int64_t k0) {
    if (TA) la.load(Ag, args.lda, k0, m0, K, M, tid);
    else    la.load(Ag, args.lda, m0, k0, M, K, tid);
    if (TB) lb.load(Bg, args.ldb, n0, k0, N, K, tid);
    else    lb.load(Bg, args.ldb, k0, n0, K, N, tid);
  };
  auto store_stage = [&](int buf) {
    la.template store<TA == 0, Cfg::LDA_S>(As + buf * Cfg::A_STAGE, tid);
    lb.template store<TB == 1, Cfg::LDB_S>(Bs + buf * Cfg::B_STAGE, tid);
  };

  // Accumulators: T*T floats per lane.
  constexpr int NACC = (T == 1) ? 4 : (T == 2) ? 4 : (T == 4) ? 16 : 64;
  float acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = 0.f;

  const int nk = (int)((K + BK - 1) / BK);
  if (nk > 0) {
    load_stage(0);
    store_stage(0);
    __syncthreads();
  }
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load_stage((int64_t)(kt + 1) * BK);
    const float* as = As + buf * Cfg::A_STAGE;
    const float* bs = Bs + buf * Cfg::B_STAGE;
    // All MFMA operands of the stage are read from LDS first, then the MFMAs
    // issue back to back (they chain on the accumulator).
    if constexpr (T == 1) {
      // 16 blocks of 4x4x1: block b = lane/4 -> output block ob = b%4 of the
      // 2x2 grid of 4x4 blocks, K offset ks = b/4.
      const int b = lane >> 2, i = lane & 3;
      const int ob = b & 3, ks = b >> 2;
      const int ar = wm0 + 4 * (ob >> 1) + i;
      const int bc = wn0 + 4 * (ob & 1) + i;
      float af[BK / 4], bf[BK / 4];
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        af[kk / 4] = as[(kk + ks) * Cfg::LDA_S + ar];
        bf[kk / 4] = bs[(kk + ks) * Cfg::LDB_S + bc];
      }
      f32x4 c = {acc[0], acc[1], acc[2], acc[3]};
#pragma unroll
      for (int q = 0; q < BK / 4; ++q) c = __builtin_amdgcn_mfma_f32_4x4x1f32(af[q], bf[q], c, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = c[r];
    } else if constexpr (T == 2) {
      const int r16 = lane & 15, kq = lane >> 4;
      float af[BK / 4], bf[BK / 4];
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        af[kk / 4] = as[(kk + kq) * Cfg::LDA_S + wm0 + r16];
        bf[kk / 4] = bs[(kk + kq) * Cfg::LDB_S + wn0 + r16];
      }
      f32x4 c = {acc[0], acc[1], acc[2], acc[3]};
#pragma unroll
      for (int q = 0; q < BK / 4; ++q) c = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q], bf[q], c, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = c[r];
    } else if constexpr (T == 4) {
      const int r32 = lane & 31, kh = lane >> 5;
      float af[BK / 2], bf[BK / 2];
#pragma unroll
      for (int kk = 0; kk < BK; kk += 2) {
        af[kk / 2] = as[(kk + kh) * Cfg::LDA_S + wm0 + r32];
        bf[kk / 2] = bs[(kk + kh) * Cfg::LDB_S + wn0 + r32];
      }
      f32x16 c;
#pragma unroll
      for (int r = 0; r < 16; ++r) c[r] = acc[r];
#pragma unroll
      for (int q = 0; q < BK / 2; ++q) c = __builtin_amdgcn_mfma_f32_32x32x2f32(af[q], bf[q], c, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = c[r];
    } else {
      const int r32 = lane & 31, kh = lane >> 5;
      f32x16 c00, c01, c10, c11;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        c00[r] = acc[r]; c01[r] = acc[16 + r]; c10[r] = acc[32 + r]; c11[r] = acc[48 + r];
      }
      // T = 8 holds 64 accumulators; operands are read a half stage at a time
      constexpr int HALF = BK / 2 > 16 ? 16 : BK / 2;
#pragma unroll
      for (int k0 = 0; k0 < BK; k0 += 2 * HALF) {
        float a0[HALF], a1[HALF], b0[HALF], b1[HALF];
#pragma unroll
        for (int q = 0; q < HALF; ++q) {
          const float* ar = as + (k0 + 2 * q + kh) * Cfg::LDA_S + wm0 + r32;
          const float* br = bs + (k0 + 2 * q + kh) * Cfg::LDB_S + wn0 + r32;
          a0[q] = ar[0]; a1[q] = ar[32];
          b0[q] = br[0]; b1[q] = br[32];
        }
#pragma unroll
        for (int q = 0; q < HALF; ++q) {
          c00 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[q], b0[q], c00, 0, 0, 0);
          c01 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[q], b1[q], c01, 0, 0, 0);
          c10 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[q], b0[q], c10, 0, 0, 0);
          c11 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[q], b1[q], c11, 0, 0, 0);
        }
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        acc[r] = c00[r]; acc[16 + r] = c01[r]; acc[32 + r] = c10[r]; acc[48 + r] = c11[r];
      }
    }
    if (kt + 1 < nk) store_stage(buf ^ 1);
    __syncthreads();
  }

  // Epilogue.
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
  if constexpr (T == 1) {
    // Sum the four K slices (lanes differing in bits 4 and 5), then lane with
    // slice s stores row s of its 4x4 block: 64 lanes store the 8x8 block.
    float s[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float v = acc[r];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      s[r] = v;
    }
    const int ob = (lane >> 2) & 3, i = lane & 3, ks = lane >> 4;
    float v = (ks == 0) ? s[0] : (ks == 1) ? s[1] : (ks == 2) ? s[2] : s[3];
    put(4 * (ob >> 1) + ks, 4 * (ob & 1) + i, v);
  } else if constexpr (T == 2) {
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

}  // namespace kt
