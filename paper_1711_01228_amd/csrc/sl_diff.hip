// Reverse mode through K unrolled iterations of Algorithm 2 (Jacobi step,
// fixed omega, the safeguard decisions of the forward run held fixed), to the
// initial placement X^0 and, for graphs with edge lengths, through the
// shortest paths to the edge lengths.
//
// One iteration, X^{k+1} = a X^H - b X with X^H = X + F(X)/W and
// (a, b) = (omega, omega - 1) if X~ was kept, else (1, 0), so a - b = 1.  With
// Gbar = dL/dX^{k+1}, g_i = a Gbar_i / W_i and, per pair (d = d_ij, r, u = (x_i -
// x_j)/r, inv = 1/d, w = inv^2):
//   dF_i/dx_i = sum_j J_ij,  dF_i/dx_j = -J_ij,  J_ij = inv (I - u u^T)/r - w I
//   dL/dX^k   = Gbar + Xbar,  Xbar_i = sum_j J_ij (g_i - g_j)
//   dL/dd_ij  (row i's use of d_ij, in F_i and W_i = sum_j w_ij)
//             = w (2 inv - 1/r) (g_i . (x_i - x_j)) - 2 w inv Wbar_i,
//   Wbar_i    = -g_i . (x^H_i - x_i) = -g_i . F_i / W_i.
// d_ij and d_ji are one variable (d is symmetric): its derivative is the sum of
// both rows' uses.  The distance of a pair s < t is the length of the tree path
// of s, so dL/dlen(u, v) collects, over the trees in which (u, v) is an edge
// with child v, the derivatives of every pair whose path runs through it:
//   delta_s(v) = sum_{t in subtree_s(v), t > s} dL/dd_st
// (dependency accumulation over each source's shortest-path tree, in the
// manner of Brandes, J. Math. Sociol. 25:163, 2001).
//
// Every sum is taken in a fixed order, so gradients are bitwise repeatable.
#include "sl_device.h"

namespace sl {

namespace {

inline unsigned blocks_for(size_t items) { return (unsigned)((items + 255) / 256); }

// Caller layout (n x dim floats) -> double columns (c * n_pad + i), 0 padding.
__global__ __launch_bounds__(256) void k_grad_in(const float* __restrict__ G, double* __restrict__ gb, int n,
                                                 int n_pad, int dim) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n_pad) return;
  for (int c = 0; c < dim; ++c) gb[(size_t)c * n_pad + i] = i < n ? (double)G[(size_t)i * dim + c] : 0.0;
}

__global__ __launch_bounds__(256) void k_grad_out(const double* __restrict__ gb, float* __restrict__ G, int n,
                                                  int n_pad, int dim) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < dim; ++c) G[(size_t)i * dim + c] = (float)gb[(size_t)c * n_pad + i];
}

// -2 F (the stress gradient, F the force-pass sums) in the caller's layout.
__global__ __launch_bounds__(256) void k_stress_grad_out(const double* __restrict__ fpart, int slices, int n,
                                                         int n_pad, int dim, float* __restrict__ G) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < dim; ++c) {
    const double f = sum_strided(fpart + (size_t)c * n_pad + i, slices, (size_t)dim * n_pad);
    G[(size_t)i * dim + c] = (float)(-2.0 * f);
  }
}

// Copy the current iterate (buffer cur of Xb) to dst.
__global__ __launch_bounds__(256) void k_save(const float* __restrict__ Xb, size_t stride,
                                              const DevState* __restrict__ st, float* __restrict__ dst) {
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= stride) return;
  dst[q] = Xb[(size_t)st->cur * stride + q];
}

// g = a Gbar / W (float, the iterate's vector layout) and Wbar = -g . F / W.
template <int DIM>
__global__ __launch_bounds__(256) void k_adj_prep(const double* __restrict__ gb, const double* __restrict__ fpart,
                                                  int slices, const double* __restrict__ W, double a, int n_pad,
                                                  float* __restrict__ gvec, float* __restrict__ wbar) {
  using V = typename VecT<DIM>::T;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n_pad) return;
  const double Wi = W[i];
  float g[3] = {0.f, 0.f, 0.f};
  double wb = 0.0;
  if (Wi > 0.0) {
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const double f = sum_strided(fpart + (size_t)c * n_pad + i, slices, (size_t)DIM * n_pad);
      const double gc = a * gb[(size_t)c * n_pad + i] / Wi;
      g[c] = (float)gc;
      wb -= gc * f / Wi;
    }
  }
  V* __restrict__ gv = reinterpret_cast<V*>(gvec);
  if constexpr (DIM == 2) gv[i] = make_float2(g[0], g[1]);
  else gv[i] = make_float4(g[0], g[1], g[2], 0.f);
  wbar[i] = (float)wb;
}

// Xbar_i = sum_j J_ij (g_i - g_j) over all ordered pairs, in the tiling of the
// force pass (one wave per row block and column slice, x_j and g_j through the
// scalar cache).  dL/dd is added per segment of iterations by k_dbar_seg.
template <int DIM, bool FD>
__global__ __launch_bounds__(256) void k_adjoint(const uint8_t* __restrict__ d, const float* __restrict__ df,
                                                 const float* __restrict__ Xk, const float* __restrict__ gvec,
                                                 double* __restrict__ apart, int nrb, int ng, int gps, int n_pad) {
  using V = typename VecT<DIM>::T;
  using C = typename DChunkT<FD>::T;
  __shared__ float2 lut[256];
  if constexpr (!FD) {
    fill_weight_table<false>(lut);
    __syncthreads();
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int rb = blockIdx.x * 4 + wave;
  if (rb >= nrb) return;
  const int slice = blockIdx.y;
  const int g0 = slice * gps;
  const int g1 = min(g0 + gps, ng);
  const V* __restrict__ X = reinterpret_cast<const V*>(Xk);
  const V* __restrict__ Gv = reinterpret_cast<const V*>(gvec);
  const int i = rb * kRowBlock + lane;
  const V xi = X[i], gi = Gv[i];
  double A0 = 0.0, A1 = 0.0, A2 = 0.0;
  for (int g = g0; g < g1; ++g) {
    const C q = load_chunk<FD>(d, df, rb, ng, g, lane);
    const V* __restrict__ xj = X + (size_t)g * kColGroup;
    const V* __restrict__ gj = Gv + (size_t)g * kColGroup;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
    for (int k = 0; k < kColGroup; ++k) {
      float inv, w;
      if constexpr (FD) {
        const float dv = fchunk_at(q, k);
        inv = dv > 0.f ? __builtin_amdgcn_rcpf(dv) : 0.f;
        w = inv * inv;
      } else {
        const float2 wt = lut[byte_of(chunk_word(q, k), k & 3)];
        inv = wt.x;
        w = wt.y;
      }
      const V p = xj[k], pg = gj[k];
      const float dx = xi.x - p.x, dy = xi.y - p.y;
      const float ex = gi.x - pg.x, ey = gi.y - pg.y;
      float r2 = fmaf(dx, dx, kTiny);
      r2 = fmaf(dy, dy, r2);
      float de = dx * ex;
      de = fmaf(dy, ey, de);
      float dz = 0.f, ez = 0.f;
      if constexpr (DIM == 3) {
        dz = xi.z - p.z;
        ez = gi.z - pg.z;
        r2 = fmaf(dz, dz, r2);
        de = fmaf(dz, ez, de);
      }
      const float rinv = __builtin_amdgcn_rsqf(r2);
      const float ir = inv * rinv;
      const float c = ir - w;
      // (inv / r^3)(d . e), ordered so that coincident points give 0, not inf * 0
      const float t = (ir * rinv) * (rinv * de);
      a0 = fmaf(c, ex, a0);
      a0 = fmaf(-t, dx, a0);
      a1 = fmaf(c, ey, a1);
      a1 = fmaf(-t, dy, a1);
      if constexpr (DIM == 3) {
        a2 = fmaf(c, ez, a2);
        a2 = fmaf(-t, dz, a2);
      }
    }
    A0 += (double)a0;
    A1 += (double)a1;
    if constexpr (DIM == 3) A2 += (double)a2;
  }
  double* ap = apart + (size_t)slice * DIM * n_pad + i;
  ap[0] = A0;
  ap[n_pad] = A1;
  if constexpr (DIM == 3) ap[2 * (size_t)n_pad] = A2;
}

// dL/dd_ij of a segment of nk iterations, added into Dbar (FP32, the tile-major
// layout of the distances: each lane rewrites its own chunk once per segment).
// Iteration m of the segment contributes, for every ordered pair,
//   w (2/d - 1/r) (g_i . (x_i - x_j)) - 2 w (1/d) Wbar_i
// with x = X^m (segX + m stride), g and Wbar the adjoint vectors of that
// iteration (gseg + m stride, wseg + m n_pad); the terms of a pair are summed
// newest first in registers.
template <int DIM, bool FD>
__global__ __launch_bounds__(256) void k_dbar_seg(const uint8_t* __restrict__ d, const float* __restrict__ df,
                                                  const float* __restrict__ segX, size_t stride,
                                                  const float* __restrict__ gseg, const float* __restrict__ wseg,
                                                  int nk, float* __restrict__ Dbar, int nrb, int ng, int gps,
                                                  int n_pad) {
  using V = typename VecT<DIM>::T;
  using C = typename DChunkT<FD>::T;
  __shared__ float2 lut[256];
  if constexpr (!FD) {
    fill_weight_table<false>(lut);
    __syncthreads();
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int rb = blockIdx.x * 4 + wave;
  if (rb >= nrb) return;
  const int g0 = blockIdx.y * gps;
  const int g1 = min(g0 + gps, ng);
  const int i = rb * kRowBlock + lane;
  for (int g = g0; g < g1; ++g) {
    const C q = load_chunk<FD>(d, df, rb, ng, g, lane);
    float inv[kColGroup], w[kColGroup], h[kColGroup];
#pragma unroll
    for (int k = 0; k < kColGroup; ++k) {
      if constexpr (FD) {
        const float dv = fchunk_at(q, k);
        inv[k] = dv > 0.f ? __builtin_amdgcn_rcpf(dv) : 0.f;
        w[k] = inv[k] * inv[k];
      } else {
        const float2 wt = lut[byte_of(chunk_word(q, k), k & 3)];
        inv[k] = wt.x;
        w[k] = wt.y;
      }
      h[k] = 0.f;
    }
    for (int m = nk - 1; m >= 0; --m) {
      const V* __restrict__ X = reinterpret_cast<const V*>(segX + (size_t)m * stride);
      const V xi = X[i];
      const V gi = reinterpret_cast<const V*>(gseg + (size_t)m * stride)[i];
      const float wbi = wseg[(size_t)m * n_pad + i];
      const V* __restrict__ xj = X + (size_t)g * kColGroup;
#pragma unroll
      for (int k = 0; k < kColGroup; ++k) {
        const V p = xj[k];
        const float dx = xi.x - p.x, dy = xi.y - p.y;
        float r2 = fmaf(dx, dx, kTiny);
        r2 = fmaf(dy, dy, r2);
        float gd = gi.x * dx;
        gd = fmaf(gi.y, dy, gd);
        if constexpr (DIM == 3) {
          const float dz = xi.z - p.z;
          r2 = fmaf(dz, dz, r2);
          gd = fmaf(gi.z, dz, gd);
        }
        const float rinv = __builtin_amdgcn_rsqf(r2);
        h[k] += w[k] * fmaf(2.f, inv[k], -rinv) * gd - 2.f * w[k] * inv[k] * wbi;
      }
    }
    float4* p = reinterpret_cast<float4*>(Dbar + ((size_t)rb * ng + g) * kTileBytes) + lane * 4;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float4 o = p[v];
      o.x += h[4 * v];
      o.y += h[4 * v + 1];
      o.z += h[4 * v + 2];
      o.w += h[4 * v + 3];
      p[v] = o;
    }
  }
}

// Gbar += Xbar (the slices of the adjoint pass).
template <int DIM>
__global__ __launch_bounds__(256) void k_adj_update(double* __restrict__ gb, const double* __restrict__ apart,
                                                    int slices, int n_pad) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n_pad) return;
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    gb[(size_t)c * n_pad + i] += sum_strided(apart + (size_t)c * n_pad + i, slices, (size_t)DIM * n_pad);
  }
}

// S[s][t] = Dbar[s][t] + Dbar[t][s] for s < t < n, row-major (stride n), from
// the tile-major Dbar, one 64 x 64 block pair (I, J >= I) per workgroup.
__global__ __launch_bounds__(256) void k_dsym(const float* __restrict__ Dbar, float* __restrict__ S, int n, int nb,
                                              int ng) {
  __shared__ float bij[4096], bji[4096];
  const int J = blockIdx.x, I = blockIdx.y;
  if (J < I || J >= nb) return;
  const float* pij = Dbar + ((size_t)I * ng + 4 * (size_t)J) * kTileBytes;
  const float* pji = Dbar + ((size_t)J * ng + 4 * (size_t)I) * kTileBytes;
  for (int e = threadIdx.x; e < 4096; e += 256) {
    bij[e] = pij[e];
    bji[e] = pji[e];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 4096; e += 256) {
    const int a = e / 64, b = e % 64;  // row a of block I, column b of block J
    const int s = I * kRowBlock + a, t = J * kRowBlock + b;
    if (s >= n || t >= n || t <= s) continue;
    const float x = bij[(b / kColGroup) * kTileBytes + a * kColGroup + b % kColGroup];
    const float y = bji[(a / kColGroup) * kTileBytes + b * kColGroup + a % kColGroup];
    S[(size_t)s * n + t] = x + y;
  }
}

// Per source s (one workgroup): delta(v) = base(v) + sum over the children c
// of v in the tree of s of delta(c), base(v) = S[s][v] for v > s, else 0.
// Children of v are its neighbours with pred = v, visited in CSR order.  The
// tree depth of every vertex comes first (rounds over the vertices in LDS, one
// per level); then the levels are taken deepest first, so each vertex scans its
// CSR row once, after all its children are final.  Leaves (most vertices of a
// shortest-path tree) keep delta = base without a scan.  Row s of S is
// replaced by delta_s.
__global__ __launch_bounds__(1024) void k_tree_accum(const int64_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col_idx,
                                                     const int32_t* __restrict__ pred, float* __restrict__ S, int n) {
  constexpr int kPer = kWeightedMaxN / 1024;
  constexpr uint16_t kUnknown = 0xffff;  // not reached (depths are below kWeightedMaxN)
  __shared__ float delta[kWeightedMaxN];
  __shared__ int16_t pr[kWeightedMaxN];
  __shared__ uint16_t depth[kWeightedMaxN];
  __shared__ uint8_t parent[kWeightedMaxN];  // v has a child in the tree
  __shared__ int changed;
  const int s = blockIdx.x;
  float base[kPer];
  int32_t rb[kPer], re[kPer];  // CSR range of each of the thread's vertices (nnz < 2^31)
  float* row = S + (size_t)s * n;
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    const int v = threadIdx.x + m * 1024;
    base[m] = (v < n && v > s) ? row[v] : 0.f;
    rb[m] = v < n ? (int32_t)row_ptr[v] : 0;
    re[m] = v < n ? (int32_t)row_ptr[v + 1] : 0;
    if (v < n) {
      delta[v] = base[m];
      pr[v] = (int16_t)pred[(size_t)s * n + v];  // -1: the source or not reached
      depth[v] = v == s ? 0 : kUnknown;
      parent[v] = 0;
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    const int v = threadIdx.x + m * 1024;
    if (v < n && pr[v] >= 0) parent[pr[v]] = 1;
  }
  // depth(v) = depth(pred(v)) + 1, one level per round
  int height = 0;
  for (int r = 1; r < n; ++r) {
    __syncthreads();
    if (threadIdx.x == 0) changed = 0;
    __syncthreads();
    bool ch = false;
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int v = threadIdx.x + m * 1024;
      if (v >= n || depth[v] != kUnknown) continue;
      const int p = pr[v];
      if (p >= 0 && depth[p] == r - 1) {
        depth[v] = (uint16_t)r;
        ch = true;
      }
    }
    if (ch) changed = 1;
    __syncthreads();
    if (!changed) break;
    height = r;
  }
  // deepest level first: the children of a vertex at level L are at level L + 1
  for (int L = height; L >= 0; --L) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int v = threadIdx.x + m * 1024;
      if (v >= n || depth[v] != L || !parent[v]) continue;
      float x = base[m];
      for (int32_t e = rb[m]; e < re[m]; e += 8) {
        int32_t cc[8];  // eight column loads in flight, then the sums in CSR order
#pragma unroll
        for (int q = 0; q < 8; ++q) cc[q] = e + q < re[m] ? col_idx[e + q] : -1;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (cc[q] >= 0 && pr[cc[q]] == v) x += delta[cc[q]];
      }
      delta[v] = x;
    }
  }
  __syncthreads();
  for (int v = threadIdx.x; v < n; v += 1024) row[v] = delta[v];
}

// G[e] for every CSR entry e = (v, u): sum over sources s, in order, of
// delta_s(v) where u is v's predecessor in the tree of s.  One workgroup per
// vertex v; thread t takes s = t, t + 256, ... into double accumulators per
// neighbour slot (32 slots a pass), summed over threads in order.
__global__ __launch_bounds__(256) void k_edge_grad(const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col_idx,
                                                   const int32_t* __restrict__ pred,
                                                   const float* __restrict__ delta, int n,
                                                   double* __restrict__ G) {
  constexpr int kSlots = 32;
  __shared__ double acc[kSlots][256];
  __shared__ int32_t nb[kSlots];
  const int v = blockIdx.x;
  const int64_t e0 = row_ptr[v], deg = row_ptr[v + 1] - e0;
  for (int64_t base = 0; base < deg; base += kSlots) {
    const int cnt = (int)min<int64_t>(kSlots, deg - base);
    __syncthreads();
    if (threadIdx.x < cnt) nb[threadIdx.x] = col_idx[e0 + base + threadIdx.x];
    for (int k = 0; k < kSlots; ++k) acc[k][threadIdx.x] = 0.0;
    __syncthreads();
    for (int s = threadIdx.x; s < n; s += 256) {
      const int32_t u = pred[(size_t)s * n + v];
      if (u < 0) continue;
      const float x = delta[(size_t)s * n + v];
      for (int k = 0; k < cnt; ++k)
        if (nb[k] == u) acc[k][threadIdx.x] += (double)x;
    }
    __syncthreads();
    if (threadIdx.x < cnt) {
      double t = 0.0;
      for (int q = 0; q < 256; ++q) t += acc[threadIdx.x][q];
      G[e0 + base + threadIdx.x] = t;
    }
  }
}

// dL/dlen of an edge = the sum of its two directed entries.
__global__ __launch_bounds__(256) void k_twin_sum(const int64_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col_idx,
                                                  const int32_t* __restrict__ erow, const double* __restrict__ G,
                                                  int64_t nnz, float* __restrict__ glen) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nnz) return;
  const int32_t v = erow[e], u = col_idx[e];
  double t = G[e];
  for (int64_t f = row_ptr[u]; f < row_ptr[u + 1]; ++f)
    if (col_idx[f] == v) t += G[f];
  glen[e] = (float)t;
}

}  // namespace

hipError_t launch_grad_in(const float* G, double* gb, int n, int n_pad, int dim, hipStream_t s) {
  k_grad_in<<<blocks_for(n_pad), 256, 0, s>>>(G, gb, n, n_pad, dim);
  return hipGetLastError();
}

hipError_t launch_grad_out(const double* gb, float* G, int n, int n_pad, int dim, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_grad_out<<<blocks_for(n), 256, 0, s>>>(gb, G, n, n_pad, dim);
  return hipGetLastError();
}

hipError_t launch_stress_grad_out(const double* fpart, int slices, int n, int n_pad, int dim, float* G,
                                  hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_stress_grad_out<<<blocks_for(n), 256, 0, s>>>(fpart, slices, n, n_pad, dim, G);
  return hipGetLastError();
}

hipError_t launch_save(const float* Xb, size_t stride, const DevState* st, float* dst, hipStream_t s) {
  k_save<<<blocks_for(stride), 256, 0, s>>>(Xb, stride, st, dst);
  return hipGetLastError();
}

hipError_t launch_adjoint_step(int dim, const uint8_t* d, const float* df, const float* Xk, const double* fpart,
                               int fslices, const double* W, double a, double* gb, float* gvec, float* wbar,
                               double* apart, const Split& sp, int n_pad, hipStream_t s) {
  const unsigned nb = blocks_for(n_pad);
  const dim3 grid(sp.blocks_x, sp.slices);
  const int gps = sp.groups_per_slice;
  // the adjoint pass overwrites fpart (the force sums were read by k_adj_prep)
  if (dim == 2) {
    k_adj_prep<2><<<nb, 256, 0, s>>>(gb, fpart, fslices, W, a, n_pad, gvec, wbar);
    if (df) k_adjoint<2, true><<<grid, 256, 0, s>>>(d, df, Xk, gvec, apart, sp.nrb, sp.ng, gps, n_pad);
    else k_adjoint<2, false><<<grid, 256, 0, s>>>(d, df, Xk, gvec, apart, sp.nrb, sp.ng, gps, n_pad);
    k_adj_update<2><<<nb, 256, 0, s>>>(gb, apart, sp.slices, n_pad);
  } else {
    k_adj_prep<3><<<nb, 256, 0, s>>>(gb, fpart, fslices, W, a, n_pad, gvec, wbar);
    if (df) k_adjoint<3, true><<<grid, 256, 0, s>>>(d, df, Xk, gvec, apart, sp.nrb, sp.ng, gps, n_pad);
    else k_adjoint<3, false><<<grid, 256, 0, s>>>(d, df, Xk, gvec, apart, sp.nrb, sp.ng, gps, n_pad);
    k_adj_update<3><<<nb, 256, 0, s>>>(gb, apart, sp.slices, n_pad);
  }
  return hipGetLastError();
}

hipError_t launch_dbar_segment(int dim, const uint8_t* d, const float* df, const float* segX, size_t stride,
                               const float* gseg, const float* wseg, int nk, float* Dbar, const Split& sp, int n_pad,
                               hipStream_t s) {
  if (nk <= 0) return hipSuccess;
  const dim3 grid(sp.blocks_x, sp.slices);
  const int gps = sp.groups_per_slice;
  if (dim == 2) {
    if (df) k_dbar_seg<2, true><<<grid, 256, 0, s>>>(d, df, segX, stride, gseg, wseg, nk, Dbar, sp.nrb, sp.ng, gps, n_pad);
    else k_dbar_seg<2, false><<<grid, 256, 0, s>>>(d, df, segX, stride, gseg, wseg, nk, Dbar, sp.nrb, sp.ng, gps, n_pad);
  } else {
    if (df) k_dbar_seg<3, true><<<grid, 256, 0, s>>>(d, df, segX, stride, gseg, wseg, nk, Dbar, sp.nrb, sp.ng, gps, n_pad);
    else k_dbar_seg<3, false><<<grid, 256, 0, s>>>(d, df, segX, stride, gseg, wseg, nk, Dbar, sp.nrb, sp.ng, gps, n_pad);
  }
  return hipGetLastError();
}

hipError_t launch_edge_grad(const float* Dbar, float* S, const int64_t* row_ptr, const int32_t* col_idx,
                            const int32_t* erow, const int32_t* pred, double* G, float* glen, int n, int64_t nnz,
                            int n_pad, int ng, hipStream_t s) {
  if (n <= 1 || nnz == 0) return hipSuccess;
  const int nb = n_pad / kRowBlock;
  k_dsym<<<dim3(nb, nb), 256, 0, s>>>(Dbar, S, n, nb, ng);
  k_tree_accum<<<n, 1024, 0, s>>>(row_ptr, col_idx, pred, S, n);
  k_edge_grad<<<n, 256, 0, s>>>(row_ptr, col_idx, pred, S, n, G);
  k_twin_sum<<<blocks_for((size_t)nnz), 256, 0, s>>>(row_ptr, col_idx, erow, G, nnz, glen);
  return hipGetLastError();
}

}  // namespace sl
