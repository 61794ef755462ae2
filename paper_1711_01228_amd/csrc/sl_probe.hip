// libslprobe: calibration of the roofline on the device at hand, for the
// benchmark (not an operation of the layout method, and not part of
// libsorlayout): the issue rate of plain FP32 FMAs (the libraries are built
// without packed FP32, so this is the vector FP32 rate the force pass can
// reach) and of the transcendentals the force and safeguard terms use (rsq,
// sqrt, rcp).  Each lane runs 8 independent chains of one instruction kind;
// 8 waves per SIMD hide the latency.
#include "slprobe.h"

#include <hip/hip_runtime.h>

#include <algorithm>

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

}  // namespace

extern "C" int32_t slp_probe_rate(int32_t kind, void* stream, double* per_s, double* ms) {
  if (!per_s || !ms) return -1;
  if (kind < 0 || kind > 3) return -1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -3;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -3;
  const int blocks = std::max(1, cus) * 8;  // 4 waves per workgroup: 8 waves per SIMD
  const int iters = 2000;
  const hipStream_t s = (hipStream_t)stream;
  float* out = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipMalloc(&out, sizeof(float) * (size_t)blocks * 256);
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = launch_probe(kind, out, blocks, iters, s);
  if (e == hipSuccess) e = hipEventRecord(a, s);
  if (e == hipSuccess) e = launch_probe(kind, out, blocks, iters, s);
  if (e == hipSuccess) e = hipEventRecord(b, s);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (out) (void)hipFree(out);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? -2 : -3;
  *ms = t;
  *per_s = (double)blocks * 256.0 * probe_ops_per_lane(iters) / (t * 1e-3);
  return 0;
}
