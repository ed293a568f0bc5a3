// Operand conversions for the low-precision GEMM paths.
//
// BF16: round to nearest even of the FP32 bit pattern, NaN kept quiet.
// FP8 e4m3 (OCP "e4m3fn", largest finite 448): per-tensor scale
// s = 448 / amax(|x|) in FP32 (s = 1 when amax = 0), code = e4m3(x * s) with
// the product rounded to FP32, round to nearest even, saturating to +-448,
// NaN -> 0x7F.  amax is an order-independent atomic maximum of the
// non-negative float bit patterns, so the scale is exact and deterministic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kt_internal.hpp"

namespace kt {

__global__ void cvt_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t u = __float_as_uint(x[i]);
    uint16_t r;
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) r = (uint16_t)((u >> 16) | 0x40u);
    else r = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
    y[i] = r;
  }
}

__global__ void zero_u32_kernel(uint32_t* p) { *p = 0u; }

__global__ void amax_kernel(const float* __restrict__ x, int64_t n, uint32_t* __restrict__ amax_bits) {
  __shared__ uint32_t red[256];
  uint32_t m = 0u;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t u = __float_as_uint(x[i]) & 0x7FFFFFFFu;   // |x| (NaN sorts above inf)
    m = u > m ? u : m;
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && red[threadIdx.x + s] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(amax_bits, red[0]);
}

__device__ __forceinline__ float fp8_scale_of(uint32_t amax_bits) {
  const float amax = __uint_as_float(amax_bits);
  return amax > 0.f ? 448.0f / amax : 1.0f;
}

__global__ void quant_fp8_kernel(const float* __restrict__ x, int64_t n,
                                 const uint32_t* __restrict__ amax_bits, uint8_t* __restrict__ y,
                                 float* __restrict__ scale_out) {
  const float s = fp8_scale_of(*amax_bits);
  if (blockIdx.x == 0 && threadIdx.x == 0) *scale_out = s;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float v = x[i] * s;
    uint8_t code;
    if (v != v) {
      code = 0x7F;
    } else {
      const float c = fminf(fmaxf(v, -448.0f), 448.0f);   // saturate, then round to nearest even
      code = (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(c, 0.0f, 0, false) & 0xFF);
    }
    y[i] = code;
  }
}

static unsigned grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace kt

using namespace kt;

extern "C" {

kt_status kt_convert_bf16(kt_handle hh, const float* x, int64_t n, uint16_t* y, void* stream) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  if (n < 0) return fail(h, KT_EINVAL, "n < 0");
  if (n == 0) return KT_OK;
  if (!x || !y) return fail(h, KT_EINVAL, "NULL buffer");
  hipLaunchKernelGGL(cvt_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, x, y, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "BF16 conversion launch");
  return KT_OK;
}

kt_status kt_quantize_fp8(kt_handle hh, const float* x, int64_t n, uint8_t* y, float* d_scale,
                          void* workspace, size_t ws_bytes, void* stream) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  if (n < 0) return fail(h, KT_EINVAL, "n < 0");
  if (!d_scale) return fail(h, KT_EINVAL, "NULL scale");
  if (n > 0 && (!x || !y)) return fail(h, KT_EINVAL, "NULL buffer");
  if (!workspace || ws_bytes < 4) return fail(h, KT_EWORKSPACE, "FP8 quantization needs 4 bytes of workspace");
  hipStream_t st = (hipStream_t)stream;
  uint32_t* amax = (uint32_t*)workspace;
  hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, st, amax);
  if (n > 0) hipLaunchKernelGGL(amax_kernel, dim3(grid_for(n)), dim3(256), 0, st, x, n, amax);
  hipLaunchKernelGGL(quant_fp8_kernel, dim3(grid_for(n)), dim3(256), 0, st, x, n,
                     (const uint32_t*)amax, y, d_scale);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "FP8 quantization launch");
  return KT_OK;
}

}  // extern "C"
