// Calibration of the roofline on the device at hand: the issue rate of plain
// FP32 FMAs (the library is built without packed FP32, so this is the vector
// FP32 rate the force pass can reach) and of the transcendentals the force and
// safeguard terms use (rsq, sqrt, rcp).  Each lane runs 8 independent chains
// of one instruction kind; 8 waves per SIMD hide the latency.
#include "sl_internal.h"

namespace sl {

namespace {

constexpr int kProbeChains = 8;
constexpr int kProbeUnroll = 16;

template <int KIND>
__global__ __launch_bounds__(256) void k_probe(float* __restrict__ out, int iters, float m, float c) {
  float a[kProbeChains];
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) a[k] = 1.0f + 1e-3f * (float)(k + 1) + 1e-7f * (float)threadIdx.x;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < kProbeUnroll; ++r) {
#pragma unroll
      for (int k = 0; k < kProbeChains; ++k) {
        if constexpr (KIND == 0) a[k] = fmaf(a[k], m, c);  // stays near c / (1 - m)
        else if constexpr (KIND == 1) a[k] = __builtin_amdgcn_rsqf(a[k]);  // fixed point 1
        else if constexpr (KIND == 2) a[k] = __builtin_amdgcn_sqrtf(a[k]);
        else a[k] = __builtin_amdgcn_rcpf(a[k]);  // a, 1/a, a, ...
      }
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) s += a[k];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

int probe_ops_per_lane(int iters) { return iters * kProbeUnroll * kProbeChains; }

hipError_t launch_probe(int kind, float* out, int blocks, int iters, hipStream_t s) {
  switch (kind) {
    case 0: k_probe<0><<<blocks, 256, 0, s>>>(out, iters, 0.999f, 1e-3f); break;
    case 1: k_probe<1><<<blocks, 256, 0, s>>>(out, iters, 0.f, 0.f); break;
    case 2: k_probe<2><<<blocks, 256, 0, s>>>(out, iters, 0.f, 0.f); break;
    default: k_probe<3><<<blocks, 256, 0, s>>>(out, iters, 0.f, 0.f); break;
  }
  return hipGetLastError();
}

}  // namespace sl
