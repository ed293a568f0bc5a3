// Seeded operand fill: a counter-based SplitMix64 hash (Steele, Lea and Flood,
// OOPSLA 2014) of (seed XOR index); the top 24 bits give a value in [-1, 1)
// that is exact in FP32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kt_internal.hpp"

namespace kt {

__device__ __forceinline__ uint64_t splitmix64_out(uint64_t s) {
  uint64_t z = s + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void fill_uniform_kernel(float* __restrict__ dst, int64_t n, uint64_t seed,
                                    int64_t offset) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint64_t h = splitmix64_out(seed ^ (uint64_t)(offset + i));
    dst[i] = (float)(uint32_t)(h >> 40) * (1.0f / 8388608.0f) - 1.0f;
  }
}

hipError_t fill_uniform(float* dst, int64_t n, uint64_t seed, int64_t offset, hipStream_t s) {
  const int64_t blocks_needed = (n + 255) / 256;
  const unsigned blocks = (unsigned)(blocks_needed < 8192 ? blocks_needed : 8192);
  hipLaunchKernelGGL(fill_uniform_kernel, dim3(blocks), dim3(256), 0, s, dst, n, seed, offset);
  return hipGetLastError();
}

}  // namespace kt
