// Ideal distances of a weighted graph: d_ij = length of a shortest path, the
// sum of edge lengths along it (Sec. 2 takes d_ij as the graph-theoretic
// distance; Sec. 5.4 lays out a net with edge lengths), in FP32, with the
// shortest-path tree of every source.
//
//   k_wsssp  one workgroup per source s, its distance row in LDS.  Rounds of
//            relaxation dist[v] = min(dist[v], min_u dist[u] + len(u, v)),
//            updated in place, until a round changes nothing: the least
//            fixpoint, i.e. for every v the smallest FP32 path sum from s
//            (lengths are positive, so shortest paths are simple).  Then
//            pred[s][v] = the lowest-numbered neighbour u with
//            dist[u] + len(u, v) == dist[v] (ties broken by the lowest id).
//   k_wsym   d_ts := d_st for s < t: the tree of the lower-numbered end
//            defines each pair, so d is symmetric bit for bit.
#include "sl_device.h"

#include <algorithm>

namespace sl {

namespace {

constexpr float kInf = __builtin_huge_valf();

__global__ __launch_bounds__(1024) void k_wsssp(const int64_t* __restrict__ row_ptr,
                                                const int32_t* __restrict__ col_idx, const float* __restrict__ len,
                                                int n, int ng, int src0, float* __restrict__ df,
                                                int32_t* __restrict__ pred) {
  __shared__ float dist[kWeightedMaxN];
  __shared__ int changed;
  const int s = src0 + blockIdx.x;
  if (s >= n) return;
  for (int v = threadIdx.x; v < n; v += blockDim.x) dist[v] = (v == s) ? 0.f : kInf;
  // a simple shortest path has at most n - 1 edges: n rounds always suffice
  for (int round = 0; round <= n; ++round) {
    __syncthreads();
    if (threadIdx.x == 0) changed = 0;
    __syncthreads();
    bool ch = false;
    for (int v = threadIdx.x; v < n; v += blockDim.x) {
      float best = dist[v];
      for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) best = fminf(best, dist[col_idx[e]] + len[e]);
      if (best < dist[v]) {
        dist[v] = best;
        ch = true;
      }
    }
    if (ch) changed = 1;
    __syncthreads();
    if (!changed) break;
  }
  __syncthreads();
  for (int v = threadIdx.x; v < n; v += blockDim.x) {
    const float dv = dist[v];
    int32_t p = -1;
    if (v != s && dv < kInf) {
      for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
        const int32_t u = col_idx[e];
        if (dist[u] + len[e] == dv && (p < 0 || u < p)) p = u;
      }
    }
    df[tile_offset(s, v, ng)] = (v != s && dv < kInf) ? dv : 0.f;
    pred[(size_t)s * n + v] = p;
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

hipError_t launch_wsssp(const int64_t* row_ptr, const int32_t* col_idx, const float* len, int n, int ng, float* df,
                        int32_t* pred, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  constexpr int kSourcesPerLaunch = 4096;
  for (int src0 = 0; src0 < n; src0 += kSourcesPerLaunch) {
    const int count = std::min(kSourcesPerLaunch, n - src0);
    k_wsssp<<<count, 1024, 0, s>>>(row_ptr, col_idx, len, n, ng, src0, df, pred);
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
