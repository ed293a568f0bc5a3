// MLP cost model: the learned selector that stands in for the decision tree
// (section 5.1 of the paper compares an MLP with its decision trees; here
// the network regresses each chosen kernel's relative performance and the
// selection is the argmax).
//
// Network 6 -> 64 -> 64 -> k, ReLU after both hidden layers, linear output,
// y = x W^T + b with W row-major [out][in].  Features of a problem:
//   [log2 M / 12, log2 N / 12, log2 K / 12, log2 batch / 6, transA, transB]
// Targets: relative performance (Q16 / 65535) of the chosen kernels.  Loss:
// mean squared error over rows x k.  Full-batch Adam with bias correction.
//
// GPU layout: one work-group per 32-row block runs forward and backward for
// its rows entirely in LDS and writes partial gradients; a second kernel sums
// the partials in block order (deterministic) and applies Adam.  A training
// run replays a captured hipGraph of several steps.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "kt_internal.hpp"

namespace kt {

static constexpr int MLP_IN = 6;
static constexpr int MLP_H = 64;
static constexpr int MLP_ROWS = 32;      // rows per work-group
static constexpr int MLP_THREADS = 256;
static constexpr int MLP_MAX_K = 64;

struct MlpLayout {
  int k;
  int oW1, ob1, oW2, ob2, oW3, ob3, total;
  __host__ __device__ explicit MlpLayout(int kk) : k(kk) {
    oW1 = 0;
    ob1 = oW1 + MLP_H * MLP_IN;
    oW2 = ob1 + MLP_H;
    ob2 = oW2 + MLP_H * MLP_H;
    oW3 = ob2 + MLP_H;
    ob3 = oW3 + kk * MLP_H;
    total = ob3 + kk;
  }
};

// log2 of a positive integer, evaluated by the same float operations on the
// host and on the device so that host and device selection agree bit for bit
// (the math libraries' log2f may differ in the last place): v = m 2^e with
// e = floor(log2 v) and m in [1, 2] (float(v) scaled exactly by 2^-e), then
// log2 m = (2 / ln 2) atanh(t), t = (m - 1) / (m + 1) in [0, 1/3], from the
// odd series t (1 + t^2/3 + ... + t^14/15) (truncation below 5e-10), in
// Horner form with explicit fused multiply-adds.  Values <= 1 give 0.
__host__ __device__ inline float feature_log2(int64_t v) {
  if (v <= 1) return 0.f;
  const int e = 63 - __builtin_clzll((unsigned long long)v);
  const float m = ldexpf((float)v, -e);
  const float t = (m - 1.f) / (m + 1.f);
  const float t2 = t * t;
  float p = 1.f / 15.f;
  p = fmaf(p, t2, 1.f / 13.f);
  p = fmaf(p, t2, 1.f / 11.f);
  p = fmaf(p, t2, 1.f / 9.f);
  p = fmaf(p, t2, 1.f / 7.f);
  p = fmaf(p, t2, 1.f / 5.f);
  p = fmaf(p, t2, 1.f / 3.f);
  p = fmaf(p, t2, 1.f);
  const float u = 2.88539008f * t;   // 2 / ln 2
  return fmaf(u, p, (float)e);
}

__host__ __device__ inline void shape_features(const kt_shape& s, float* x) {
  x[0] = feature_log2(s.M) * (1.0f / 12.0f);
  x[1] = feature_log2(s.N) * (1.0f / 12.0f);
  x[2] = feature_log2(s.K) * (1.0f / 12.0f);
  x[3] = feature_log2(s.batch) * (1.0f / 6.0f);
  x[4] = (float)s.transA;
  x[5] = (float)s.transB;
}

// Features -> forward -> argmax (lowest index on ties): the position in the
// chosen list.  Shared by the batch selection kernel and the host launcher
// path, with the same operation order, so both pick the same kernel.
__host__ __device__ inline int mlp_forward_argmax(const kt_shape& shape, const float* P, int k) {
  const MlpLayout L(k);
  float x[MLP_IN], h1[MLP_H], h2[MLP_H];
  shape_features(shape, x);
  for (int o = 0; o < MLP_H; ++o) {
    float s = P[L.ob1 + o];
    for (int q = 0; q < MLP_IN; ++q) s = fmaf(x[q], P[L.oW1 + o * MLP_IN + q], s);
    h1[o] = fmaxf(s, 0.f);
  }
  for (int o = 0; o < MLP_H; ++o) {
    float s = P[L.ob2 + o];
    for (int q = 0; q < MLP_H; ++q) s = fmaf(h1[q], P[L.oW2 + o * MLP_H + q], s);
    h2[o] = fmaxf(s, 0.f);
  }
  int best = 0;
  float bv = 0.f;
  for (int o = 0; o < k; ++o) {
    float s = P[L.ob3 + o];
    for (int q = 0; q < MLP_H; ++q) s = fmaf(h2[q], P[L.oW3 + o * MLP_H + q], s);
    if (o == 0 || s > bv) { bv = s; best = o; }
  }
  return best;
}

__global__ void mlp_features_kernel(const kt_shape* __restrict__ shapes, int n, float* __restrict__ X) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) shape_features(shapes[i], X + (int64_t)i * MLP_IN);
}

// Targets: Y[i][j] = q[i][chosen[j]] / 65535 from the normalized table.
__global__ void mlp_targets_kernel(const uint16_t* __restrict__ Xq, int n, int d,
                                   const int32_t* __restrict__ chosen, int k, float* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * k) return;
  const int64_t i = e / k;
  const int j = (int)(e % k);
  Y[e] = (float)Xq[i * d + chosen[j]] * (1.0f / 65535.0f);
}

// Forward and backward of one block of MLP_ROWS rows.  Writes the block's
// partial gradient (same layout as the parameters) and partial sum of
// squared errors; optionally the predictions.  step: block 0 increments the
// Adam step counter.  Weight rows sit in LDS with an odd stride (7, 65) so
// that the 64 lanes of a wave, which read one column of 64 different rows,
// hit 64 different banks.
static constexpr int W1S = MLP_IN + 1;     // LDS row strides of W1, W2, W3
static constexpr int W2S = MLP_H + 1;
static constexpr int W3S = MLP_H + 1;

__global__ void __launch_bounds__(MLP_THREADS)
mlp_fwdbwd_kernel(const float* __restrict__ P, const float* __restrict__ X, const float* __restrict__ Y,
                  int n, int k, float* __restrict__ part, float* __restrict__ part_loss,
                  float* __restrict__ pred, int* __restrict__ step) {
  extern __shared__ float sm[];
  const MlpLayout L(k);
  float* W1 = sm;                                  // [64][W1S]
  float* W2 = W1 + MLP_H * W1S;                    // [64][W2S]
  float* W3 = W2 + MLP_H * W2S;                    // [k][W3S]
  float* b1 = W3 + MLP_MAX_K * W3S;                // [64]
  float* b2 = b1 + MLP_H;                          // [64]
  float* b3 = b2 + MLP_H;                          // [k]
  float* xs = b3 + MLP_MAX_K;                      // [ROWS][6]
  float* z1 = xs + MLP_ROWS * MLP_IN;              // [ROWS][64]  z1
  float* z2 = z1 + MLP_ROWS * MLP_H;               // [ROWS][64]  z2, later dz1
  float* yy = z2 + MLP_ROWS * MLP_H;               // [ROWS][MAX_K] dy
  float* dh = yy + MLP_ROWS * MLP_MAX_K;           // [ROWS][64]  dz2
  __shared__ float red[MLP_THREADS];
  const int tid = threadIdx.x;
  const int r0 = blockIdx.x * MLP_ROWS;
  const int rows = min(MLP_ROWS, n - r0);
  if (blockIdx.x == 0 && tid == 0 && step) *step += 1;
  for (int e = tid; e < MLP_H * MLP_IN; e += MLP_THREADS) W1[(e / MLP_IN) * W1S + e % MLP_IN] = P[L.oW1 + e];
  for (int e = tid; e < MLP_H * MLP_H; e += MLP_THREADS) W2[(e / MLP_H) * W2S + e % MLP_H] = P[L.oW2 + e];
  for (int e = tid; e < k * MLP_H; e += MLP_THREADS) W3[(e / MLP_H) * W3S + e % MLP_H] = P[L.oW3 + e];
  for (int e = tid; e < MLP_H; e += MLP_THREADS) { b1[e] = P[L.ob1 + e]; b2[e] = P[L.ob2 + e]; }
  for (int e = tid; e < k; e += MLP_THREADS) b3[e] = P[L.ob3 + e];
  for (int e = tid; e < MLP_ROWS * MLP_IN; e += MLP_THREADS) {
    const int r = e / MLP_IN;
    xs[e] = r < rows ? X[(int64_t)(r0 + r) * MLP_IN + e % MLP_IN] : 0.f;
  }
  __syncthreads();
  // z1 = x W1^T + b1          (lane -> output unit o)
  for (int e = tid; e < MLP_ROWS * MLP_H; e += MLP_THREADS) {
    const int r = e / MLP_H, o = e % MLP_H;
    float s = b1[o];
    for (int i = 0; i < MLP_IN; ++i) s = fmaf(xs[r * MLP_IN + i], W1[o * W1S + i], s);
    z1[e] = s;
  }
  __syncthreads();
  // z2 = relu(z1) W2^T + b2
  for (int e = tid; e < MLP_ROWS * MLP_H; e += MLP_THREADS) {
    const int r = e / MLP_H, o = e % MLP_H;
    float s = b2[o];
    for (int i = 0; i < MLP_H; ++i) s = fmaf(fmaxf(z1[r * MLP_H + i], 0.f), W2[o * W2S + i], s);
    z2[e] = s;
  }
  __syncthreads();
  // y = relu(z2) W3^T + b3 ; dy = 2 (y - Y) / (n k) ; loss partial
  const float scale = 2.0f / ((float)n * (float)k);
  float lsum = 0.f;
  for (int e = tid; e < MLP_ROWS * k; e += MLP_THREADS) {
    const int r = e / k, o = e % k;
    float s = b3[o];
    for (int i = 0; i < MLP_H; ++i) s = fmaf(fmaxf(z2[r * MLP_H + i], 0.f), W3[o * W3S + i], s);
    float dy = 0.f;
    if (r < rows) {
      if (pred) pred[(int64_t)(r0 + r) * k + o] = s;
      if (Y) {
        const float diff = s - Y[(int64_t)(r0 + r) * k + o];
        lsum = fmaf(diff, diff, lsum);
        dy = scale * diff;
      }
    }
    yy[r * MLP_MAX_K + o] = dy;
  }
  red[tid] = lsum;
  __syncthreads();
  for (int s = MLP_THREADS / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (!part) return;   // inference only (uniform across the block)
  if (tid == 0) part_loss[blockIdx.x] = red[0];
  float* g = part + (int64_t)blockIdx.x * L.total;
  // dW3[o][i] = sum_r dy[r][o] relu(z2[r][i]);  db3[o] = sum_r dy[r][o]   (lane -> i)
  for (int e = tid; e < k * MLP_H; e += MLP_THREADS) {
    const int o = e / MLP_H, i = e % MLP_H;
    float s = 0.f;
    for (int r = 0; r < MLP_ROWS; ++r) s = fmaf(yy[r * MLP_MAX_K + o], fmaxf(z2[r * MLP_H + i], 0.f), s);
    g[L.oW3 + e] = s;
  }
  for (int o = tid; o < k; o += MLP_THREADS) {
    float s = 0.f;
    for (int r = 0; r < MLP_ROWS; ++r) s += yy[r * MLP_MAX_K + o];
    g[L.ob3 + o] = s;
  }
  // dz2 = (dy W3) * [z2 > 0]    (lane -> i)
  for (int e = tid; e < MLP_ROWS * MLP_H; e += MLP_THREADS) {
    const int r = e / MLP_H, i = e % MLP_H;
    float s = 0.f;
    for (int o = 0; o < k; ++o) s = fmaf(yy[r * MLP_MAX_K + o], W3[o * W3S + i], s);
    dh[e] = z2[e] > 0.f ? s : 0.f;
  }
  __syncthreads();
  // dW2[o][i] = sum_r dz2[r][o] relu(z1[r][i]); db2       (lane -> i)
  for (int e = tid; e < MLP_H * MLP_H; e += MLP_THREADS) {
    const int o = e / MLP_H, i = e % MLP_H;
    float s = 0.f;
    for (int r = 0; r < MLP_ROWS; ++r) s = fmaf(dh[r * MLP_H + o], fmaxf(z1[r * MLP_H + i], 0.f), s);
    g[L.oW2 + e] = s;
  }
  for (int o = tid; o < MLP_H; o += MLP_THREADS) {
    float s = 0.f;
    for (int r = 0; r < MLP_ROWS; ++r) s += dh[r * MLP_H + o];
    g[L.ob2 + o] = s;
  }
  // dz1 = (dz2 W2) * [z1 > 0], written over z2 (no longer needed)   (lane -> i)
  for (int e = tid; e < MLP_ROWS * MLP_H; e += MLP_THREADS) {
    const int r = e / MLP_H, i = e % MLP_H;
    float s = 0.f;
    for (int o = 0; o < MLP_H; ++o) s = fmaf(dh[r * MLP_H + o], W2[o * W2S + i], s);
    z2[e] = z1[e] > 0.f ? s : 0.f;
  }
  __syncthreads();
  // dW1[o][i] = sum_r dz1[r][o] x[r][i]; db1
  for (int e = tid; e < MLP_H * MLP_IN; e += MLP_THREADS) {
    const int o = e / MLP_IN, i = e % MLP_IN;
    float s = 0.f;
    for (int r = 0; r < MLP_ROWS; ++r) s = fmaf(z2[r * MLP_H + o], xs[r * MLP_IN + i], s);
    g[L.oW1 + e] = s;
  }
  for (int o = tid; o < MLP_H; o += MLP_THREADS) {
    float s = 0.f;
    for (int r = 0; r < MLP_ROWS; ++r) s += z2[r * MLP_H + o];
    g[L.ob1 + o] = s;
  }
}

// Sum the block partials in block order; optionally write the gradient and
// loss, and optionally apply one Adam step (t read from *step).
__global__ void mlp_reduce_adam_kernel(float* __restrict__ P, const float* __restrict__ part,
                                       const float* __restrict__ part_loss, int nblocks, int total,
                                       float* __restrict__ grad_out, float* __restrict__ loss_out,
                                       float* __restrict__ m, float* __restrict__ v,
                                       const int* __restrict__ step, float lr, int adam) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0 && loss_out) {
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += part_loss[b];
    *loss_out = s;   // sum of squared errors; the mean is this / (n k)
  }
  if (e >= total) return;
  float gsum = 0.f;
  for (int b = 0; b < nblocks; ++b) gsum += part[(int64_t)b * total + e];
  if (grad_out) grad_out[e] = gsum;
  if (adam) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const int t = *step;
    const float mm = b1 * m[e] + (1.f - b1) * gsum;
    const float vv = b2 * v[e] + (1.f - b2) * gsum * gsum;
    m[e] = mm;
    v[e] = vv;
    const float c1 = 1.f - powf(b1, (float)t);
    const float c2 = 1.f - powf(b2, (float)t);
    P[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  }
}

// Batch selection: features -> forward -> argmax (lowest index on ties) -> id.
__global__ void mlp_select_kernel(const kt_shape* __restrict__ shapes, int n, const float* __restrict__ P,
                                  int k, const int32_t* __restrict__ chosen, int32_t* __restrict__ ids) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  ids[i] = chosen[mlp_forward_argmax(shapes[i], P, k)];
}

static size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

struct MlpPlan {
  size_t oP, oM, oV, oG, oPart, oPL, oX, oY, oStep, oLoss, oShapes, oT, oQ, oChosen, total;
  int nblocks;
};

static MlpPlan mlp_plan(int n, int k, int d) {
  MlpPlan p;
  const MlpLayout L(k);
  p.nblocks = (n + MLP_ROWS - 1) / MLP_ROWS;
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o = a256(o + bytes); return at; };
  p.oP = take((size_t)L.total * 4);
  p.oM = take((size_t)L.total * 4);
  p.oV = take((size_t)L.total * 4);
  p.oG = take((size_t)L.total * 4);
  p.oPart = take((size_t)p.nblocks * L.total * 4);
  p.oPL = take((size_t)p.nblocks * 4);
  p.oX = take((size_t)n * MLP_IN * 4);
  p.oY = take((size_t)n * k * 4);
  p.oStep = take(4);
  p.oLoss = take(4);
  p.oShapes = take((size_t)n * sizeof(kt_shape));
  p.oT = take((size_t)n * d * 8);
  p.oQ = take((size_t)n * d * 2);
  p.oChosen = take((size_t)k * 4);
  p.total = o;
  return p;
}

static size_t fwdbwd_lds(int k) {
  (void)k;
  return ((size_t)MLP_H * (MLP_IN + 1) + MLP_H * (MLP_H + 1) + MLP_MAX_K * (MLP_H + 1) + 2 * MLP_H +
          MLP_MAX_K + MLP_ROWS * MLP_IN + 2 * MLP_ROWS * MLP_H + MLP_ROWS * MLP_MAX_K +
          MLP_ROWS * MLP_H) * 4;
}

static hipError_t launch_fwdbwd(const float* P, const float* X, const float* Y, int n, int k,
                                float* part, float* part_loss, float* pred, int* step, hipStream_t st) {
  const int nb = (n + MLP_ROWS - 1) / MLP_ROWS;
  hipLaunchKernelGGL(mlp_fwdbwd_kernel, dim3(nb), dim3(MLP_THREADS), fwdbwd_lds(k), st, P, X, Y, n,
                     k, part, part_loss, pred, step);
  return hipGetLastError();
}

static hipError_t set_lds_attr(int k) {
  return hipFuncSetAttribute((const void*)mlp_fwdbwd_kernel,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)fwdbwd_lds(k));
}

// He-uniform initialisation U(+-sqrt(6 / fan_in)) from SplitMix64(seed),
// W1, W2, W3 in that order, row-major; zero biases.
static void he_uniform(std::vector<float>& P, int k, uint64_t seed) {
  const MlpLayout L(k);
  P.assign(L.total, 0.f);
  uint64_t state = seed;
  auto next_uniform = [&]() {
    uint64_t z = state + 0x9E3779B97F4A7C15ull;
    state = z;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
  };
  auto fill = [&](int off, int fan_out, int fan_in) {
    const double bound = sqrt(6.0 / fan_in);
    for (int e = 0; e < fan_out * fan_in; ++e) P[off + e] = (float)((2.0 * next_uniform() - 1.0) * bound);
  };
  fill(L.oW1, MLP_H, MLP_IN);
  fill(L.oW2, MLP_H, MLP_H);
  fill(L.oW3, k, MLP_H);
}

kt_status mlp_upload(Ctx* h, int dtype) {
  SelState& S = h->sel[dtype];
  if (h->device < 0) return KT_OK;
  if (S.d_mlp) { (void)hipFree(S.d_mlp); S.d_mlp = nullptr; }
  const size_t pbytes = S.mlp.params.size() * 4, cbytes = S.chosen.size() * 4;
  hipError_t e = hipMalloc(&S.d_mlp, pbytes + cbytes + 256);
  if (e != hipSuccess) { S.d_mlp = nullptr; return hip_fail(h, e, "hipMalloc MLP weights"); }
  e = hipMemcpy(S.d_mlp, S.mlp.params.data(), pbytes, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy((char*)S.d_mlp + pbytes, S.chosen.data(), cbytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(h, e, "upload MLP weights");
  return KT_OK;
}

kt_status mlp_select_batch(Ctx* h, int dtype, const kt_shape* d_shapes, int32_t n, int32_t* d_ids,
                           hipStream_t st) {
  SelState& S = h->sel[dtype];
  if (!S.d_mlp) return fail(h, KT_ENOTFITTED, "MLP weights not on the device");
  const int k = S.mlp.k;
  const float* P = (const float*)S.d_mlp;
  const int32_t* chosen = (const int32_t*)((const char*)S.d_mlp + S.mlp.params.size() * 4);
  hipLaunchKernelGGL(mlp_select_kernel, dim3((n + 63) / 64), dim3(64), 0, st, d_shapes, n, P, k,
                     chosen, d_ids);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "MLP select launch");
  return KT_OK;
}

// Host selection: the same forward pass on the host copy of the weights, so
// kt_gemm(config_id = -1) with the MLP selector makes no device call besides
// the GEMM launch itself (no copy, no synchronization, capturable in a graph).
kt_status mlp_select_host(Ctx* h, int dtype, const kt_shape* s, int32_t* id) {
  const SelState& S = h->sel[dtype];
  if (S.mlp.params.empty() || S.mlp.k < 1) return fail(h, KT_ENOTFITTED, "no MLP weights");
  *id = S.chosen[mlp_forward_argmax(*s, S.mlp.params.data(), S.mlp.k)];
  return KT_OK;
}

kt_status fit_mlp(Ctx* h, int dtype, const kt_shape* shapes, const int64_t* time_ns, int32_t n,
                  int32_t d, const int32_t* chosen, int32_t k, const kt_mlp_opts* o, void* ws,
                  size_t ws_bytes, hipStream_t st) {
  if (!need_device(h)) return KT_EINVAL;
  if (k > MLP_MAX_K) return fail(h, KT_EINVAL, "MLP supports k <= 64");
  kt_mlp_opts opts = {3000, 1e-3f, nullptr, 13150, 25};
  if (o) opts = *o;
  if (opts.steps < 0 || opts.graph_steps < 0) return fail(h, KT_EINVAL, "negative step count");
  const MlpPlan p = mlp_plan(n, k, d);
  if (!ws || ws_bytes < p.total) return fail(h, KT_EWORKSPACE, "MLP workspace too small");
  char* w = (char*)ws;
  const MlpLayout L(k);
  std::vector<float> P0;
  if (opts.init) P0.assign(opts.init, opts.init + L.total);
  else he_uniform(P0, k, opts.seed);
  hipError_t e = hipMemcpyAsync(w + p.oP, P0.data(), (size_t)L.total * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(w + p.oM, 0, (size_t)L.total * 4, st);
  if (e == hipSuccess) e = hipMemsetAsync(w + p.oV, 0, (size_t)L.total * 4, st);
  if (e == hipSuccess) e = hipMemsetAsync(w + p.oStep, 0, 4, st);
  if (e == hipSuccess) e = hipMemcpyAsync(w + p.oShapes, shapes, (size_t)n * sizeof(kt_shape), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(w + p.oT, time_ns, (size_t)n * d * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(w + p.oChosen, chosen, (size_t)k * 4, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(h, e, "MLP upload");
  kt_status s = kt_normalize(reinterpret_cast<kt_handle>(h), (const int64_t*)(w + p.oT), n, d,
                             KT_NORM_RELATIVE, (uint16_t*)(w + p.oQ), st);
  if (s != KT_OK) return s;
  hipLaunchKernelGGL(mlp_features_kernel, dim3((n + 255) / 256), dim3(256), 0, st,
                     (const kt_shape*)(w + p.oShapes), n, (float*)(w + p.oX));
  hipLaunchKernelGGL(mlp_targets_kernel, dim3((unsigned)(((int64_t)n * k + 255) / 256)), dim3(256), 0, st,
                     (const uint16_t*)(w + p.oQ), n, d, (const int32_t*)(w + p.oChosen), k,
                     (float*)(w + p.oY));
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(h, e, "MLP data kernels");
  if ((e = set_lds_attr(k)) != hipSuccess) return hip_fail(h, e, "MLP LDS attribute");
  float* P = (float*)(w + p.oP);
  auto one_step = [&](hipStream_t s2) -> hipError_t {
    hipError_t r = launch_fwdbwd(P, (const float*)(w + p.oX), (const float*)(w + p.oY), n, k,
                                 (float*)(w + p.oPart), (float*)(w + p.oPL), nullptr, (int*)(w + p.oStep), s2);
    if (r != hipSuccess) return r;
    hipLaunchKernelGGL(mlp_reduce_adam_kernel, dim3((L.total + 255) / 256), dim3(256), 0, s2, P,
                       (const float*)(w + p.oPart), (const float*)(w + p.oPL), p.nblocks, L.total,
                       nullptr, nullptr, (float*)(w + p.oM), (float*)(w + p.oV),
                       (const int*)(w + p.oStep), opts.lr, 1);
    return hipGetLastError();
  };
  int done = 0;
  if (opts.graph_steps > 1 && opts.steps >= opts.graph_steps) {
    // Capture graph_steps steps once and replay the graph.
    hipStream_t cs = st;
    bool own = false;
    if (cs == nullptr) {
      if ((e = hipStreamCreate(&cs)) != hipSuccess) return hip_fail(h, e, "capture stream");
      own = true;
      if ((e = hipStreamSynchronize(nullptr)) != hipSuccess) return hip_fail(h, e, "sync");
    }
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    for (int i = 0; i < opts.graph_steps && e == hipSuccess; ++i) e = one_step(cs);
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    while (e == hipSuccess && opts.steps - done >= opts.graph_steps) {
      e = hipGraphLaunch(exec, cs);
      done += opts.graph_steps;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (own) {
      if (e == hipSuccess) e = hipStreamSynchronize(cs);
      (void)hipStreamDestroy(cs);
    }
    if (e != hipSuccess) return hip_fail(h, e, "MLP training graph");
  }
  for (; done < opts.steps; ++done)
    if ((e = one_step(st)) != hipSuccess) return hip_fail(h, e, "MLP training step");
  std::vector<float> trained(L.total);
  e = hipMemcpyAsync(trained.data(), P, (size_t)L.total * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(h, e, "read MLP weights");
  free_selector_device(h, dtype);
  SelState& S = h->sel[dtype];
  S = SelState();
  S.mlp.k = k;
  S.mlp.params = std::move(trained);
  S.chosen.assign(chosen, chosen + k);
  return mlp_upload(h, dtype);
}

}  // namespace kt

using namespace kt;

extern "C" {

kt_status kt_mlp_workspace_bytes(int32_t n_rows, int32_t n_configs, int32_t k, size_t* bytes) {
  if (!bytes || n_rows < 1 || n_configs < 1 || k < 1 || k > MLP_MAX_K) return KT_EINVAL;
  *bytes = mlp_plan(n_rows, k, n_configs).total;
  return KT_OK;
}

kt_status kt_mlp_num_params(int32_t k, int32_t* n_params) {
  if (!n_params || k < 1 || k > MLP_MAX_K) return KT_EINVAL;
  *n_params = MlpLayout(k).total;
  return KT_OK;
}

kt_status kt_mlp_features(kt_handle hh, const kt_shape* d_shapes, int32_t n, float* d_X, void* stream) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  if (n < 0) return fail(h, KT_EINVAL, "n < 0");
  if (n == 0) return KT_OK;
  if (!d_shapes || !d_X) return fail(h, KT_EINVAL, "NULL argument");
  hipLaunchKernelGGL(mlp_features_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                     d_shapes, n, d_X);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "features launch");
  return KT_OK;
}

kt_status kt_mlp_forward_backward(kt_handle hh, const float* d_params, const float* d_X,
                                  const float* d_Y, int32_t n, int32_t k, float* d_pred,
                                  float* d_grad, float* d_loss, void* ws, size_t ws_bytes,
                                  void* stream) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  if (n < 1 || k < 1 || k > MLP_MAX_K) return fail(h, KT_EINVAL, "need n >= 1 and 1 <= k <= 64");
  if (!d_params || !d_X) return fail(h, KT_EINVAL, "NULL argument");
  if ((d_grad || d_loss) && !d_Y) return fail(h, KT_EINVAL, "gradients need targets");
  const MlpLayout L(k);
  const int nb = (n + MLP_ROWS - 1) / MLP_ROWS;
  const size_t need = a256((size_t)nb * L.total * 4) + a256((size_t)nb * 4);
  if ((d_grad || d_loss) && (!ws || ws_bytes < need)) return fail(h, KT_EWORKSPACE, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = set_lds_attr(k);
  if (e != hipSuccess) return hip_fail(h, e, "MLP LDS attribute");
  float* part = (d_grad || d_loss) ? (float*)ws : nullptr;
  float* pl = part ? (float*)((char*)ws + a256((size_t)nb * L.total * 4)) : nullptr;
  e = launch_fwdbwd(d_params, d_X, (d_grad || d_loss) ? d_Y : nullptr, n, k, part, pl, d_pred, nullptr, st);
  if (e != hipSuccess) return hip_fail(h, e, "forward/backward launch");
  if (part) {
    hipLaunchKernelGGL(mlp_reduce_adam_kernel, dim3((L.total + 255) / 256), dim3(256), 0, st,
                       (float*)nullptr, (const float*)part, (const float*)pl, nb, L.total, d_grad,
                       d_loss, (float*)nullptr, (float*)nullptr, (const int*)nullptr, 0.f, 0);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "gradient reduction launch");
  }
  return KT_OK;
}

kt_status kt_get_mlp(kt_handle hh, kt_dtype dtype, int32_t* n_params, float* params) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if ((int)dtype < 0 || (int)dtype >= NUM_DTYPES) return fail(h, KT_EINVAL, "bad dtype");
  if (!n_params) return fail(h, KT_EINVAL, "NULL n_params");
  const SelState& S = h->sel[dtype];
  if (S.kind != KT_SEL_MLP) return fail(h, KT_ENOTFITTED, "no MLP fitted");
  *n_params = (int32_t)S.mlp.params.size();
  if (params) memcpy(params, S.mlp.params.data(), S.mlp.params.size() * 4);
  return KT_OK;
}

}  // extern "C"
