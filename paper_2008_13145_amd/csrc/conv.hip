// Convolution layers computed through the selected GEMMs (section 6 runs a
// VGG16 network whose convolutions and fully connected layers are matrix
// multiplications).  Activations are NHWC, filters (R, S, Cin, Cout), FP32.
//
// IM2COL: every output position p = (b, i, j) becomes one row of a
// P x (R*S*Cin) matrix whose columns run over (r, s, c) with c fastest; the
// product with the filter viewed as (R*S*Cin) x Cout is the NHWC output.
//
// WINOGRAD (F(2x2, 3x3), Lavin and Gray 2016; 3x3 filters, stride 1): each
// 2x2 output tile needs a 4x4 input tile d; V = Bt d B and U = G g Gt are
// formed for every tile / channel pair, the 16 elementwise products summed
// over channels are 16 independent T x Cin by Cin x Cout GEMMs (one batched
// launch of batch 16), and Y = At M A gives the 2x2 outputs.
//   Bt = [1 0 -1 0; 0 1 1 0; 0 -1 1 0; 0 1 0 -1]
//   G  = [1 0 0; 1/2 1/2 1/2; 1/2 -1/2 1/2; 0 0 1]
//   At = [1 1 1 0; 0 1 -1 -1]
//
// Transform kernels are HBM-bound; each thread owns one channel (or output
// channel) of one row / tile, so loads and stores run along the contiguous C
// dimension.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kt_internal.hpp"

namespace kt {

namespace {

constexpr int CT = 256;            // threads per work-group of the transform kernels
constexpr unsigned MAX_GRID = 65536;

unsigned grid_for(int64_t work_groups) {
  return (unsigned)(work_groups < (int64_t)MAX_GRID ? (work_groups > 0 ? work_groups : 1) : MAX_GRID);
}

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

struct ConvDims {
  int64_t n, H, W, C, O, Ho, Wo;
  int32_t R, S, st, pad;
};

// One work-group per output row p (grid-stride); threads over the R*S*C columns.
__global__ void __launch_bounds__(CT)
im2col_kernel(const float* __restrict__ x, ConvDims d, float* __restrict__ col) {
  const int64_t P = d.n * d.Ho * d.Wo;
  const int64_t RSC = (int64_t)d.R * d.S * d.C;
  for (int64_t p = blockIdx.x; p < P; p += gridDim.x) {
    const int64_t b = p / (d.Ho * d.Wo);
    const int64_t rem = p - b * d.Ho * d.Wo;
    const int64_t i = rem / d.Wo, j = rem - (rem / d.Wo) * d.Wo;
    float* out = col + p * RSC;
    for (int64_t q = threadIdx.x; q < RSC; q += CT) {
      const int64_t rs = q / d.C, c = q - rs * d.C;
      const int64_t r = rs / d.S, s = rs - r * d.S;
      const int64_t yi = i * d.st - d.pad + r, xj = j * d.st - d.pad + s;
      float v = 0.f;
      if (yi >= 0 && yi < d.H && xj >= 0 && xj < d.W) v = x[((b * d.H + yi) * d.W + xj) * d.C + c];
      out[q] = v;
    }
  }
}

// y[r][o] = act(y[r][o] + bias[o]) over rows x O.
__global__ void __launch_bounds__(CT)
bias_act_kernel(float* __restrict__ y, int64_t rows, int64_t O, const float* __restrict__ bias,
                int32_t relu) {
  const int64_t total = rows * O;
  for (int64_t e = (int64_t)blockIdx.x * CT + threadIdx.x; e < total; e += (int64_t)gridDim.x * CT) {
    float v = y[e];
    if (bias) v += bias[e % O];
    y[e] = relu ? fmaxf(v, 0.f) : v;
  }
}

// V[k][t][c], k = 4u + v, for tile t = (b, ty, tx) and channel c.
__global__ void __launch_bounds__(CT)
wino_input_kernel(const float* __restrict__ x, ConvDims d, int64_t tH, int64_t tW,
                  float* __restrict__ V) {
  const int64_t T = d.n * tH * tW;
  const int64_t total = T * d.C;
  for (int64_t e = (int64_t)blockIdx.x * CT + threadIdx.x; e < total; e += (int64_t)gridDim.x * CT) {
    const int64_t t = e / d.C, c = e - t * d.C;
    const int64_t b = t / (tH * tW);
    const int64_t rem = t - b * tH * tW;
    const int64_t ty = rem / tW, tx = rem - ty * tW;
    const int64_t y0 = 2 * ty - d.pad, x0 = 2 * tx - d.pad;
    float v[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int64_t yi = y0 + u, xj = x0 + w;
        v[u][w] = (yi >= 0 && yi < d.H && xj >= 0 && xj < d.W)
                      ? x[((b * d.H + yi) * d.W + xj) * d.C + c] : 0.f;
      }
    float r[4][4];   // Bt d
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      r[0][w] = v[0][w] - v[2][w];
      r[1][w] = v[1][w] + v[2][w];
      r[2][w] = v[2][w] - v[1][w];
      r[3][w] = v[1][w] - v[3][w];
    }
    const int64_t plane = T * d.C;
    float* out = V + t * d.C + c;
#pragma unroll
    for (int u = 0; u < 4; ++u) {   // (Bt d) B
      out[(4 * u + 0) * plane] = r[u][0] - r[u][2];
      out[(4 * u + 1) * plane] = r[u][1] + r[u][2];
      out[(4 * u + 2) * plane] = r[u][2] - r[u][1];
      out[(4 * u + 3) * plane] = r[u][1] - r[u][3];
    }
  }
}

// U[k][c][o] = (G g Gt)[k] for the 3x3 filter g = w[:, :, c, o].
__global__ void __launch_bounds__(CT)
wino_filter_kernel(const float* __restrict__ w, int64_t C, int64_t O, float* __restrict__ U) {
  const int64_t total = C * O;
  for (int64_t e = (int64_t)blockIdx.x * CT + threadIdx.x; e < total; e += (int64_t)gridDim.x * CT) {
    float g[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int s = 0; s < 3; ++s) g[r][s] = w[(int64_t)(r * 3 + s) * total + e];
    float a[4][3];   // G g
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      a[0][s] = g[0][s];
      a[1][s] = 0.5f * (g[0][s] + g[1][s] + g[2][s]);
      a[2][s] = 0.5f * (g[0][s] - g[1][s] + g[2][s]);
      a[3][s] = g[2][s];
    }
    float* out = U + e;
#pragma unroll
    for (int u = 0; u < 4; ++u) {   // (G g) Gt
      out[(4 * u + 0) * total] = a[u][0];
      out[(4 * u + 1) * total] = 0.5f * (a[u][0] + a[u][1] + a[u][2]);
      out[(4 * u + 2) * total] = 0.5f * (a[u][0] - a[u][1] + a[u][2]);
      out[(4 * u + 3) * total] = a[u][2];
    }
  }
}

// Y = At M A per tile and output channel, plus bias and activation.
__global__ void __launch_bounds__(CT)
wino_output_kernel(const float* __restrict__ Mm, ConvDims d, int64_t tH, int64_t tW,
                   const float* __restrict__ bias, int32_t relu, float* __restrict__ y) {
  const int64_t T = d.n * tH * tW;
  const int64_t total = T * d.O;
  const int64_t plane = total;
  for (int64_t e = (int64_t)blockIdx.x * CT + threadIdx.x; e < total; e += (int64_t)gridDim.x * CT) {
    const int64_t t = e / d.O, o = e - t * d.O;
    float m[4][4];
#pragma unroll
    for (int k = 0; k < 16; ++k) m[k / 4][k % 4] = Mm[k * plane + e];
    float r[2][4];   // At M
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      r[0][w] = m[0][w] + m[1][w] + m[2][w];
      r[1][w] = m[1][w] - m[2][w] - m[3][w];
    }
    const int64_t b = t / (tH * tW);
    const int64_t rem = t - b * tH * tW;
    const int64_t ty = rem / tW, tx = rem - ty * tW;
    const float bo = bias ? bias[o] : 0.f;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const float out2[2] = {r[u][0] + r[u][1] + r[u][2], r[u][1] - r[u][2] - r[u][3]};
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        const int64_t i = 2 * ty + u, j = 2 * tx + w;
        if (i < d.Ho && j < d.Wo) {
          const float v = out2[w] + bo;
          y[((b * d.Ho + i) * d.Wo + j) * d.O + o] = relu ? fmaxf(v, 0.f) : v;
        }
      }
    }
  }
}

__global__ void __launch_bounds__(CT)
maxpool2x2_kernel(const float* __restrict__ x, int64_t n, int64_t H, int64_t W, int64_t C,
                  float* __restrict__ y) {
  const int64_t Ho = H / 2, Wo = W / 2;
  const int64_t total = n * Ho * Wo * C;
  for (int64_t e = (int64_t)blockIdx.x * CT + threadIdx.x; e < total; e += (int64_t)gridDim.x * CT) {
    const int64_t c = e % C;
    const int64_t q = e / C;
    const int64_t j = q % Wo, i = (q / Wo) % Ho, b = q / (Wo * Ho);
    const float* p = x + ((b * H + 2 * i) * W + 2 * j) * C + c;
    const float v = fmaxf(fmaxf(p[0], p[C]), fmaxf(p[W * C], p[W * C + C]));
    y[e] = v;
  }
}

kt_status check_conv(Ctx* h, kt_conv_algo algo, const kt_conv_shape* c, ConvDims* d) {
  if (!c) return fail(h, KT_EINVAL, "conv shape is NULL");
  if (algo != KT_CONV_IM2COL && algo != KT_CONV_WINOGRAD && algo != KT_CONV_WINOGRAD_PRETRANSFORMED)
    return fail(h, KT_EINVAL, "bad algorithm");
  if (c->n < 0 || c->H < 0 || c->W < 0 || c->Cin < 1 || c->Cout < 1)
    return fail(h, KT_EINVAL, "need n, H, W >= 0 and Cin, Cout >= 1");
  if (c->R < 1 || c->S < 1 || c->stride < 1 || c->pad < 0)
    return fail(h, KT_EINVAL, "need R, S, stride >= 1 and pad >= 0");
  if (algo != KT_CONV_IM2COL && (c->R != 3 || c->S != 3 || c->stride != 1))
    return fail(h, KT_EUNSUPPORTED, "Winograd F(2x2,3x3) needs a 3x3 filter and stride 1");
  d->n = c->n; d->H = c->H; d->W = c->W; d->C = c->Cin; d->O = c->Cout;
  d->R = c->R; d->S = c->S; d->st = c->stride; d->pad = c->pad;
  const int64_t hh = c->H + 2 * (int64_t)c->pad - c->R, ww = c->W + 2 * (int64_t)c->pad - c->S;
  d->Ho = hh < 0 ? 0 : hh / c->stride + 1;
  d->Wo = ww < 0 ? 0 : ww / c->stride + 1;
  return KT_OK;
}

void conv_gemm_shape(const ConvDims& d, kt_conv_algo algo, kt_shape* s) {
  s->transA = 0;
  s->transB = 0;
  s->N = d.O;
  if (algo == KT_CONV_IM2COL) {
    s->M = d.n * d.Ho * d.Wo;
    s->K = (int64_t)d.R * d.S * d.C;
    s->batch = 1;
  } else {
    s->M = d.n * ((d.Ho + 1) / 2) * ((d.Wo + 1) / 2);
    s->K = d.C;
    s->batch = 16;
  }
}

// A 1x1 filter with stride 1 and no padding: the patch matrix is x itself.
bool pointwise(const ConvDims& d) { return d.R == 1 && d.S == 1 && d.st == 1 && d.pad == 0; }

// Patch matrix (im2col, none for pointwise layers) or transforms (Winograd).
size_t conv_main_bytes(const ConvDims& d, kt_conv_algo algo) {
  kt_shape s;
  conv_gemm_shape(d, algo, &s);
  if (algo == KT_CONV_IM2COL) return pointwise(d) ? 0 : a256((size_t)s.M * s.K * 4);
  const size_t u = algo == KT_CONV_WINOGRAD ? a256((size_t)16 * d.C * d.O * 4) : 0;
  return a256((size_t)16 * s.M * d.C * 4) + u + a256((size_t)16 * s.M * d.O * 4);
}

kt_status check_splits(Ctx* h, kt_conv_algo algo, int32_t splits) {
  if (splits < 0 || splits > 64) return fail(h, KT_EINVAL, "need 0 <= splits <= 64");
  if (algo != KT_CONV_IM2COL && splits > 1)
    return fail(h, KT_EUNSUPPORTED, "split-K is offered for the im2col lowering only");
  return KT_OK;
}

// Total workspace: the main part, then the split-K partial planes.
kt_status conv_ws_bytes(Ctx* h, const ConvDims& d, kt_conv_algo algo, int32_t splits, size_t* out) {
  size_t extra = 0;
  if (algo == KT_CONV_IM2COL && splits != 1) {
    kt_shape s;
    conv_gemm_shape(d, algo, &s);
    kt_status st = kt_gemm_splitk_workspace_bytes(&s, splits, &extra);
    if (st != KT_OK) return fail(h, st, "split-K workspace query");
  }
  *out = conv_main_bytes(d, algo) + extra;
  return KT_OK;
}

}  // namespace

}  // namespace kt

using namespace kt;

extern "C" {

kt_status kt_conv2d_gemm_shape(const kt_conv_shape* c, kt_conv_algo algo, kt_shape* out) {
  ConvDims d;
  if (!out) return fail(nullptr, KT_EINVAL, "out is NULL");
  kt_status st = check_conv(nullptr, algo, c, &d);
  if (st != KT_OK) return st;
  conv_gemm_shape(d, algo, out);
  return KT_OK;
}

kt_status kt_conv2d_workspace_bytes(const kt_conv_shape* c, kt_conv_algo algo, int32_t splits,
                                    size_t* bytes) {
  ConvDims d;
  if (!bytes) return fail(nullptr, KT_EINVAL, "bytes is NULL");
  kt_status st = check_conv(nullptr, algo, c, &d);
  if (st == KT_OK) st = check_splits(nullptr, algo, splits);
  if (st != KT_OK) return st;
  return conv_ws_bytes(nullptr, d, algo, splits, bytes);
}

kt_status kt_conv2d(kt_handle hh, kt_conv_algo algo, const kt_conv_shape* c, const float* x,
                    const float* w, const float* bias, int32_t relu, float* y, int32_t config_id,
                    int32_t splits, void* workspace, size_t ws_bytes, void* stream) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  ConvDims d;
  kt_status st = check_conv(h, algo, c, &d);
  if (st == KT_OK) st = check_splits(h, algo, splits);
  if (st != KT_OK) return st;
  if (d.n == 0 || d.Ho == 0 || d.Wo == 0) return KT_OK;
  if (!x || !w || !y) return fail(h, KT_EINVAL, "x, w or y is NULL");
  size_t need = 0;
  if ((st = conv_ws_bytes(h, d, algo, splits, &need)) != KT_OK) return st;
  if (need > 0 && (!workspace || ws_bytes < need))
    return fail(h, KT_EWORKSPACE, "conv workspace too small");
  if (config_id >= (int32_t)h->configs[KT_F32].size())
    return fail(h, KT_EINVAL, "config id out of range");
  kt_shape gs;
  conv_gemm_shape(d, algo, &gs);
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  hipError_t e;
  if (algo == KT_CONV_IM2COL) {
    const float* col = x;
    if (!pointwise(d)) {
      hipLaunchKernelGGL(im2col_kernel, dim3(grid_for(gs.M)), dim3(CT), 0, s, x, d, (float*)ws);
      if ((e = hipGetLastError()) != hipSuccess) return hip_fail(h, e, "im2col launch");
      col = (const float*)ws;
    }
    // y (P x O) = col (P x RSC) * w (RSC x O)
    bool fused = false;   // bias and activation applied by the split-K reduction
    if (splits == 1) {
      int32_t cfg = config_id;
      int32_t sel = -1;
      if (cfg < 0) {
        if ((st = select_config(h, KT_F32, &gs, &sel)) != KT_OK) return st;
        cfg = kernel_base(h, KT_F32, sel);
      }
      const size_t planes = sel >= 0 ? kernel_plane_bytes(h, KT_F32, &gs, sel) : 0;
      if (planes > 0 && h->gemm_ws && h->gemm_ws_bytes >= planes) {
        // a selected split-K kernel runs split, its planes in the handle's
        // workspace, and its reduction applies the bias and the activation
        st = splitk_gemm(h, KT_F32, &gs, kernel_slices(h, KT_F32, sel), 1.f, col, gs.K,
                         gs.M * gs.K, w, d.O, gs.K * d.O, 0.f, y, d.O, gs.M * d.O, nullptr,
                         nullptr, cfg, h->gemm_ws, h->gemm_ws_bytes, stream, nullptr, bias, relu,
                         &fused);
      } else {
        st = launch_gemm(h, KT_F32, &gs, 1.f, col, gs.K, gs.M * gs.K, w, d.O, gs.K * d.O, 0.f, y,
                         d.O, gs.M * d.O, nullptr, nullptr, cfg, s);
      }
    } else {
      const size_t main = conv_main_bytes(d, algo);
      st = splitk_gemm(h, KT_F32, &gs, splits, 1.f, col, gs.K, gs.M * gs.K, w, d.O, gs.K * d.O,
                       0.f, y, d.O, gs.M * d.O, nullptr, nullptr, config_id, ws + main,
                       ws_bytes - main, stream, nullptr, bias, relu, &fused);
    }
    if (st != KT_OK) return st;
    if ((bias || relu) && !fused) {
      hipLaunchKernelGGL(bias_act_kernel, dim3(grid_for(cdiv(gs.M * d.O, CT))), dim3(CT), 0, s, y,
                         gs.M, d.O, bias, relu);
      if ((e = hipGetLastError()) != hipSuccess) return hip_fail(h, e, "bias launch");
    }
    return KT_OK;
  }
  int32_t cfg = config_id;
  if (cfg < 0) {
    if ((st = select_config(h, KT_F32, &gs, &cfg)) != KT_OK) return st;
    cfg = kernel_base(h, KT_F32, cfg);
  }
  const int64_t tH = (d.Ho + 1) / 2, tW = (d.Wo + 1) / 2, T = gs.M;
  const bool pre = algo == KT_CONV_WINOGRAD_PRETRANSFORMED;   // w already holds U
  float* V = (float*)ws;
  char* after_v = ws + a256((size_t)16 * T * d.C * 4);
  const float* U = pre ? w : (const float*)after_v;
  float* Mm = (float*)(pre ? after_v : after_v + a256((size_t)16 * d.C * d.O * 4));
  hipLaunchKernelGGL(wino_input_kernel, dim3(grid_for(cdiv(T * d.C, CT))), dim3(CT), 0, s, x, d,
                     tH, tW, V);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(h, e, "Winograd input launch");
  if (!pre) {
    hipLaunchKernelGGL(wino_filter_kernel, dim3(grid_for(cdiv(d.C * d.O, CT))), dim3(CT), 0, s, w,
                       d.C, d.O, (float*)after_v);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(h, e, "Winograd filter launch");
  }
  // M[k] (T x O) = V[k] (T x C) * U[k] (C x O), k = 0..15
  st = launch_gemm(h, KT_F32, &gs, 1.f, V, d.C, T * d.C, U, d.O, d.C * d.O, 0.f, Mm, d.O, T * d.O,
                   nullptr, nullptr, cfg, s);
  if (st != KT_OK) return st;
  hipLaunchKernelGGL(wino_output_kernel, dim3(grid_for(cdiv(T * d.O, CT))), dim3(CT), 0, s, Mm, d,
                     tH, tW, bias, relu, y);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(h, e, "Winograd output launch");
  return KT_OK;
}

kt_status kt_winograd_filter(kt_handle hh, const float* w, int64_t Cin, int64_t Cout, float* U,
                             void* stream) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  if (Cin < 1 || Cout < 1) return fail(h, KT_EINVAL, "need Cin, Cout >= 1");
  if (!w || !U) return fail(h, KT_EINVAL, "w or U is NULL");
  hipLaunchKernelGGL(wino_filter_kernel, dim3(grid_for(cdiv(Cin * Cout, CT))), dim3(CT), 0,
                     (hipStream_t)stream, w, Cin, Cout, U);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "Winograd filter launch");
  return KT_OK;
}

kt_status kt_maxpool2x2(kt_handle hh, const float* x, int64_t n, int64_t H, int64_t W, int64_t C,
                        float* y, void* stream) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  if (n < 0 || H < 0 || W < 0 || C < 0) return fail(h, KT_EINVAL, "negative size");
  const int64_t total = n * (H / 2) * (W / 2) * C;
  if (total == 0) return KT_OK;
  if (!x || !y) return fail(h, KT_EINVAL, "x or y is NULL");
  hipLaunchKernelGGL(maxpool2x2_kernel, dim3(grid_for(cdiv(total, CT))), dim3(CT), 0,
                     (hipStream_t)stream, x, n, H, W, C, y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "max-pool launch");
  return KT_OK;
}

}  // extern "C"
