// Device-side fill with the SplitMix64 counter generator (Steele, Lea, Flood,
// OOPSLA 2014): cell (i, j) of an n-column grid gets output k = i*n + j of the
// stream seeded with `seed`, mapped exactly as wfgen/__init__.py maps it
// (float32: (x >> 40) * 2^-24; float64: (x >> 11) * 2^-53; int32: x & 255).  Input
// generation only.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void fill_kernel(void* dst, int dtype, int64_t rows, int64_t n, int64_t ld, uint64_t seed, int64_t row0) {
  const int64_t total = rows * n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int64_t i = t / n, j = t - i * n;
    const uint64_t x = splitmix64_at(seed, (uint64_t)(row0 + i) * (uint64_t)n + (uint64_t)j);
    if (dtype == 0) ((float*)dst)[i * ld + j] = (float)(x >> 40) * 5.9604644775390625e-08f;  // 2^-24, exact
    else if (dtype == 2) ((double*)dst)[i * ld + j] = (double)(x >> 11) * 1.1102230246251565e-16;  // 2^-53, exact
    else ((int32_t*)dst)[i * ld + j] = (int32_t)(x & 255u);
  }
}

}  // namespace

// Fill rows [row0, row0 + rows) of an n-column grid into dst (row stride ld elements).
// dtype: 0 = float32, 1 = int32, 2 = float64.  Returns 0 or a hipError_t value.
extern "C" int wfgen_fill(void* dst, int dtype, int64_t rows, int64_t n, int64_t ld, uint64_t seed, int64_t row0,
                          void* stream) {
  if (rows <= 0 || n <= 0) return 0;
  if (!dst || ld < n || dtype < 0 || dtype > 2) return (int)hipErrorInvalidValue;
  int64_t blocks = (rows * n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, dst, dtype, rows, n, ld,
                     seed, row0);
  return (int)hipGetLastError();
}
