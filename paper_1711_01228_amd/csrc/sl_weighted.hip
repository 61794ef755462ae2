// Ideal distances of a weighted graph: d_ij = length of a shortest path, the
// sum of edge lengths along it (Sec. 2 takes d_ij as the graph-theoretic
// distance; Sec. 5.4 lays out a net with edge lengths), in FP32, with the
// shortest-path tree of every source.
//
//   k_wsssp  one workgroup per source s, its distance row in LDS.  Rounds of
//            relaxation dist[v] = min(dist[v], dist[u] + len(u, v)) over every
//            CSR entry (v, u), edge-parallel (consecutive threads take
//            consecutive entries; the minimum is an LDS atomic on the bit
//            pattern, which orders non-negative floats as unsigned integers),
//            in place, until a round improves nothing: the least fixpoint,
//            i.e. for every v the smallest FP32 path sum from s (lengths are
//            positive, so shortest paths are simple), whatever the order of
//            the updates.  Then pred[s][v] = the lowest-numbered neighbour u
//            with dist[u] + len(u, v) == dist[v] (an LDS atomic minimum on u).
//   k_wsym   d_ts := d_st for s < t: the tree of the lower-numbered end
//            defines each pair, so d is symmetric bit for bit.
#include "sl_device.h"

#include <algorithm>
#include <cstdint>

namespace sl {

namespace {

constexpr float kInf = __builtin_huge_valf();

__global__ __launch_bounds__(1024) void k_wsssp(const int32_t* __restrict__ erow, const int32_t* __restrict__ col_idx,
                                                const float* __restrict__ len, int64_t nnz, int n, int ng, int src0,
                                                float* __restrict__ df, int32_t* __restrict__ pred) {
  __shared__ uint32_t dist[kWeightedMaxN];  // FP32 bit patterns
  __shared__ int32_t pr[kWeightedMaxN];
  __shared__ int changed;
  const int s = src0 + blockIdx.x;
  if (s >= n) return;
  const uint32_t kInfBits = __float_as_uint(kInf);
  for (int v = threadIdx.x; v < n; v += blockDim.x) {
    dist[v] = (v == s) ? 0u : kInfBits;
    pr[v] = INT32_MAX;
  }
  // a simple shortest path has at most n - 1 edges: n rounds always suffice
  for (int round = 0; round <= n; ++round) {
    __syncthreads();
    if (threadIdx.x == 0) changed = 0;
    __syncthreads();
    bool ch = false;
#pragma unroll 4
    for (int64_t e = threadIdx.x; e < nnz; e += blockDim.x) {
      const int32_t v = erow[e], u = col_idx[e];
      const float du = __uint_as_float(dist[u]);
      const float cand = du + len[e];
      if (cand < __uint_as_float(dist[v])) {  // inf + len stays inf and never passes
        atomicMin(&dist[v], __float_as_uint(cand));
        ch = true;
      }
    }
    if (ch) changed = 1;
    __syncthreads();
    if (!changed) break;
  }
  __syncthreads();
#pragma unroll 4
  for (int64_t e = threadIdx.x; e < nnz; e += blockDim.x) {
    const int32_t v = erow[e], u = col_idx[e];
    const float dv = __uint_as_float(dist[v]);
    if (v != s && dv < kInf && __uint_as_float(dist[u]) + len[e] == dv) atomicMin(&pr[v], u);
  }
  __syncthreads();
  for (int v = threadIdx.x; v < n; v += blockDim.x) {
    const float dv = __uint_as_float(dist[v]);
    const bool reach = v != s && dv < kInf;
    df[tile_offset(s, v, ng)] = reach ? dv : 0.f;
    pred[(size_t)s * n + v] = reach ? pr[v] : -1;
  }
}

// Copy the upper triangle onto the lower one, one 64 x 64 block pair per
// workgroup: block (I, J), J >= I, is staged in LDS and written transposed
// into block (J, I) (on the diagonal only below it).  A block of rows I and
// column groups 4J .. 4J+3 is 4096 contiguous floats of the tile-major layout.
__global__ __launch_bounds__(256) void k_wsym(float* __restrict__ df, int nb, int ng) {
  __shared__ float blk[4096];
  const int J = blockIdx.x, I = blockIdx.y;
  if (J < I || J >= nb) return;
  const float* src = df + ((size_t)I * ng + 4 * (size_t)J) * kTileBytes;
  float* dst = df + ((size_t)J * ng + 4 * (size_t)I) * kTileBytes;
  for (int e = threadIdx.x; e < 4096; e += 256) blk[e] = src[e];
  __syncthreads();
  for (int e = threadIdx.x; e < 4096; e += 256) {
    // element e of block (J, I): row a (in J), column b (in I)
    const int a = (e / kColGroup) % kRowBlock, b = (e / kTileBytes) * kColGroup + e % kColGroup;
    if (I == J && a <= b) continue;  // keep the diagonal and the upper triangle
    dst[e] = blk[(a / kColGroup) * kTileBytes + b * kColGroup + a % kColGroup];
  }
}

}  // namespace

hipError_t launch_wsssp(const int32_t* erow, const int32_t* col_idx, const float* len, int64_t nnz, int n, int ng,
                        float* df, int32_t* pred, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  constexpr int kSourcesPerLaunch = 4096;
  for (int src0 = 0; src0 < n; src0 += kSourcesPerLaunch) {
    const int count = std::min(kSourcesPerLaunch, n - src0);
    k_wsssp<<<count, 1024, 0, s>>>(erow, col_idx, len, nnz, n, ng, src0, df, pred);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_wsym(float* df, int n_pad, int ng, hipStream_t s) {
  const int nb = n_pad / kRowBlock;
  k_wsym<<<dim3(nb, nb), 256, 0, s>>>(df, nb, ng);
  return hipGetLastError();
}

}  // namespace sl
