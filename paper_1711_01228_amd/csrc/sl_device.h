// Device helpers shared by the single-graph kernels (sl_kernels.hip) and the
// batched kernels (sl_batch.hip).
#pragma once

#include "sl_internal.h"

namespace sl {

template <int DIM> struct VecT;
template <> struct VecT<2> { using T = float2; };
template <> struct VecT<3> { using T = float4; };

// Added to r^2 so that rsq never sees 0: for coincident vertices (or i = j)
// the pair term is c * (x_i - x_j) = c * 0 = 0 with c finite.
constexpr float kTiny = 1e-30f;

__device__ __forceinline__ uint32_t chunk_word(const uint4& q, int k) {
  return (k < 4) ? q.x : (k < 8) ? q.y : (k < 12) ? q.z : q.w;
}

// sum over s = 0, 1, ..., count - 1 of a[s * stride], added in that order, with
// eight loads in flight (the partial sums of one vertex over column slices)
__device__ __forceinline__ double sum_strided(const double* __restrict__ a, int count, size_t stride) {
  double t = 0.0;
  int s = 0;
  for (; s + 8 <= count; s += 8) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = a[(size_t)(s + q) * stride];
#pragma unroll
    for (int q = 0; q < 8; ++q) t += v[q];
  }
  for (; s < count; ++s) t += a[(size_t)s * stride];
  return t;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic tree sum of K doubles over a 256-thread block.  Thread 0 gets
// the totals in v.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double (*sh)[256]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < K; ++k) sh[k][t] = v[k];
  __syncthreads();
  for (int s = 128; s >= 1; s >>= 1) {
    if (t < s) {
#pragma unroll
      for (int k = 0; k < K; ++k) sh[k][t] += sh[k][t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = sh[k][0];
  }
}

// Per-block table of the weights a distance byte stands for, built in LDS at
// kernel start: entry b holds 1/b and 1/b^2 (correctly rounded), and 1 in .z
// for the stress terms; entry 0 (same vertex, no path, padding) is all zero.
template <bool STRESS> struct WeightEntry { using T = float2; };
template <> struct WeightEntry<true> { using T = float4; };

template <bool STRESS>
__device__ __forceinline__ void fill_weight_table(typename WeightEntry<STRESS>::T* lut) {
  for (int b = threadIdx.x; b < 256; b += blockDim.x) {
    const float fb = (float)b;
    const float inv = b ? 1.0f / fb : 0.f;
    const float w = b ? 1.0f / (fb * fb) : 0.f;
    if constexpr (STRESS) lut[b] = make_float4(inv, w, b ? 1.f : 0.f, 0.f);
    else lut[b] = make_float2(inv, w);
  }
}

// Deterministic sum of K doubles over a block of W waves: a butterfly inside
// each wave, then thread k adds the W wave totals of value k in wave order.
// Every thread gets the totals in v.  sh holds K x W doubles, tot K doubles.
template <int K, int W>
__device__ __forceinline__ void block_sum_waves(double (&v)[K], double (*sh)[W], double* tot) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) sh[k][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double t = 0.0;
    for (int w = 0; w < W; ++w) t += sh[threadIdx.x][w];
    tot[threadIdx.x] = t;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = tot[k];
}

// 0xff in byte b of the result for every set bit b of the nibble.
__device__ __forceinline__ uint32_t byte_mask4(uint32_t nib) {
  return ((nib & 1u) ? 0x000000ffu : 0u) | ((nib & 2u) ? 0x0000ff00u : 0u) | ((nib & 4u) ? 0x00ff0000u : 0u) |
         ((nib & 8u) ? 0xff000000u : 0u);
}

__device__ __forceinline__ uint32_t byte_of(uint32_t word, int b) { return (word >> (8 * b)) & 0xffu; }

// ---------------------------------------------------------------------------
// Distance storage.  Hop counts are bytes (a lane chunk of 16 columns is one
// uint4); lengths of weighted graphs are floats in the same tile-major order
// (a lane chunk is 64 bytes, four float4).  0 stands for the same vertex, no
// path or padding in both.
// ---------------------------------------------------------------------------
struct FChunk {
  float4 a, b, c, e;
};

template <bool FD> struct DChunkT { using T = uint4; };
template <> struct DChunkT<true> { using T = FChunk; };

__device__ __forceinline__ float fchunk_at(const FChunk& q, int k) {
  const float4& v = (k < 4) ? q.a : (k < 8) ? q.b : (k < 12) ? q.c : q.e;
  switch (k & 3) {
    case 0: return v.x;
    case 1: return v.y;
    case 2: return v.z;
    default: return v.w;
  }
}

// The lane chunk of row block rb, column group g (d: bytes, df: floats).
template <bool FD>
__device__ __forceinline__ typename DChunkT<FD>::T load_chunk(const uint8_t* __restrict__ d,
                                                              const float* __restrict__ df, int rb, int ng, int g,
                                                              int lane) {
  if constexpr (FD) {
    const float4* p = reinterpret_cast<const float4*>(df + ((size_t)rb * ng + g) * kTileBytes) + lane * 4;
    return FChunk{p[0], p[1], p[2], p[3]};
  } else {
    return reinterpret_cast<const uint4*>(d + ((size_t)rb * ng + g) * kTileBytes)[lane];
  }
}

template <bool FD>
__device__ __forceinline__ typename DChunkT<FD>::T zero_chunk() {
  if constexpr (FD) {
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    return FChunk{z, z, z, z};
  } else {
    return make_uint4(0u, 0u, 0u, 0u);
  }
}

// Distance k of a chunk as a float (bytes: the hop count).
template <bool FD>
__device__ __forceinline__ float chunk_dist(const typename DChunkT<FD>::T& q, int k) {
  if constexpr (FD) return fchunk_at(q, k);
  else return (float)byte_of(chunk_word(q, k), k & 3);
}

}  // namespace sl
