// wf_seed.hip -- device generation of seeded serving inputs (WF_INPUT_SEED).
//
// Cell (i, j) of an m x n request gets output k = i*n + j of the SplitMix64
// stream seeded with `seed` (Steele, Lea and Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014): z = seed + (k+1)*0x9E3779B97F4A7C15,
// then the published 64-bit finaliser.  float32 cells take the top 24 bits
// scaled by 2^-24 (uniform on [0, 1), exact); int32 cells the low 8 bits.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wfk {
namespace {

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void seed_fill_kernel(uint32_t* dst, int dtype, int64_t total, uint64_t seed) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += stride) {
    const uint64_t x = splitmix64(seed, (uint64_t)k);
    dst[k] = dtype == 0 ? __builtin_bit_cast(uint32_t, (float)(uint32_t)(x >> 40) * 0x1p-24f) : (uint32_t)(x & 255u);
  }
}

}  // namespace

// Fill a dense m x n block (row stride n) on `stream`.
hipError_t launch_seed_fill(void* dst, int dtype, int64_t m, int64_t n, uint64_t seed, hipStream_t stream) {
  const int64_t total = m * n;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(seed_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, (uint32_t*)dst, dtype, total, seed);
  return hipGetLastError();
}

}  // namespace wfk
