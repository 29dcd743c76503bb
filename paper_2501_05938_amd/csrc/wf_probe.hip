// wf_probe.hip -- the latency floor of the sweep's walk, measured on the device.
//
// One wave runs the walk's per-step dependency chain with nothing else around it:
// N moves one lane down by DPP (wave_shr:1), then H = c + min(N, NW, H), one fp32
// add after an exact min.  Every step depends on the previous one, so the time per
// step is the latency of that chain; m + n - 1 such steps are the shortest possible
// sweep of an m x n grid by lanes that each own a row.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wfk {
namespace {

__device__ __forceinline__ float shr1(float old, float src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                               __builtin_bit_cast(int, src), 0x138, 0xf, 0xf, false));
}

__global__ void __launch_bounds__(64) chain_kernel(float* out, uint64_t* ticks, int steps) {
  const int lane = threadIdx.x;
  float H = (float)lane * 0.001f, Np = 0.0f;
  const float c = 1.0f / (float)(lane + 1), top = 0.5f;
  const uint64_t t0 = wall_clock64();
  for (int i = 0; i < steps; i += 16) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const float N = shr1(top, H);
      H = c + __builtin_fminf(__builtin_fminf(N, Np), H);
      Np = N;
    }
  }
  const uint64_t t1 = wall_clock64();
  out[lane] = H;
  if (lane == 0) ticks[0] = t1 - t0;
}

}  // namespace

hipError_t launch_chain_probe(float* out, uint64_t* ticks, int steps, hipStream_t stream) {
  hipLaunchKernelGGL(chain_kernel, dim3(1), dim3(64), 0, stream, out, ticks, steps);
  return hipGetLastError();
}

}  // namespace wfk
