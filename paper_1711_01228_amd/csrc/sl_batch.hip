// Batched layouts for gfx950: thousands of small graphs (n <= 1024) laid out
// by one persistent launch.  Each workgroup takes the next graph from a queue
// ordered largest first, keeps its iterates, weights and force partials in
// LDS, and runs Algorithm 2 for that graph to its own termination test: the
// same arithmetic as the single-graph kernels (force pass, Jacobi update and
// extrapolation of eq. 11, safeguard of Alg. 2 summed inside the pass
// that takes the next force at X~, residual test), with workgroup barriers in
// place of kernel boundaries.  Distances come from a
// per-graph breadth-first search run the same way.
#include "sl_device.h"

#include <algorithm>
#include <type_traits>

namespace sl {

namespace {

// ---------------------------------------------------------------------------
// Distances and weights, one graph per workgroup.  256 sources per sweep, one
// bit each in 4 words per vertex, frontiers in LDS; a thread per vertex pulls
// its neighbours' frontier words (the batch graphs have small degrees: the
// first kNbr neighbours of each of the thread's vertices stay in registers for
// the whole graph, the others are read from a copy of the graph's column
// indices in LDS when they fit, so that no level waits on global memory).  The
// sweep's 256 distance bytes of each of the thread's rows are built in
// registers and written once, as whole 16-byte chunks of the tile-major block,
// when the sweep ends.  W_v = sum_j d_vj^-2 is summed as the levels are found:
// a level l adds (new sources) / l^2, in the order sweep, level, word.
// ---------------------------------------------------------------------------
template <int T>
__global__ __launch_bounds__(T) void k_batch_distances(const BatchGraph* __restrict__ graphs,
                                                       const int32_t* __restrict__ order, int count,
                                                       int32_t* __restrict__ queue, const int64_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col_idx, uint8_t* __restrict__ d,
                                                       double* __restrict__ Wg, int32_t* __restrict__ status) {
  constexpr int kWords = 4;
  constexpr int kPer = kBatchMaxN / T;  // vertices per thread: v = tid + r T
  constexpr int kNbr = 8;               // neighbours per vertex held in registers
  constexpr int kLdsEntries = 8192;     // CSR entries of a graph kept in LDS
  __shared__ uint64_t fa[kBatchMaxN * kWords], fb[kBatchMaxN * kWords], vis[kBatchMaxN * kWords];
  __shared__ int32_t cols[kLdsEntries];
  __shared__ double wl[256];
  __shared__ int sh_q, sh_found[3];
  const int tid = threadIdx.x;
  for (int b = tid; b < 256; b += T) wl[b] = b ? 1.0 / ((double)b * (double)b) : 0.0;
  for (;;) {
    __syncthreads();
    if (tid == 0) sh_q = atomicAdd(queue, 1);
    __syncthreads();
    const int q = sh_q;
    if (q >= count) break;
    const int gid = order[q];
    const BatchGraph G = graphs[gid];
    const int n = G.n, ng = G.n_pad / kColGroup;
    uint8_t* __restrict__ dg = d + G.d_off;
    int err = 0;
    // the graph's column indices (local ids) in LDS when they fit
    const int64_t ebase = row_ptr[G.v_off], nnz = row_ptr[G.v_off + n] - ebase;
    const bool in_lds = nnz <= kLdsEntries;
    if (in_lds)
      for (int e = tid; e < (int)nnz; e += T) cols[e] = (int)(col_idx[ebase + e] - G.v_off);
    // the thread's rows: degree, first CSR entry, first kNbr neighbours, W sum
    int deg[kPer], nb[kPer][kNbr];
    int64_t e0[kPer];
    double ws[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int v = tid + r * T;
      deg[r] = 0;
      e0[r] = 0;
      ws[r] = 0.0;
      if (v < n) {
        e0[r] = row_ptr[G.v_off + v];
        deg[r] = (int)(row_ptr[G.v_off + v + 1] - e0[r]);
      }
#pragma unroll
      for (int j = 0; j < kNbr; ++j) nb[r][j] = j < deg[r] ? (int)(col_idx[e0[r] + j] - G.v_off) : 0;
    }
    for (int base = 0; base < n && !err; base += 64 * kWords) {
      // byt[r][k][c][m]: bytes 4 m .. 4 m + 3 of the 16-byte chunk of sources
      // base + 64 k + 16 c .. + 15 in row tid + r T
      uint32_t byt[kPer][kWords][4][4];
#pragma unroll
      for (int r = 0; r < kPer; ++r)
#pragma unroll
        for (int k = 0; k < kWords; ++k)
#pragma unroll
          for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int m = 0; m < 4; ++m) byt[r][k][c][m] = 0u;
      for (int v = tid; v < n; v += T) {
#pragma unroll
        for (int k = 0; k < kWords; ++k) {
          const int s0 = base + 64 * k;
          const uint64_t w = (v >= s0 && v < s0 + 64) ? (1ull << (v - s0)) : 0ull;
          fa[v * kWords + k] = w;
          vis[v * kWords + k] = w;
        }
      }
      uint64_t* F = fa;
      uint64_t* N = fb;
      if (tid < 3) sh_found[tid] = 0;
      __syncthreads();
      // One barrier per level.  sh_found[l % 3] is set by every thread that
      // finds a new pair at level l and read by all after the level's barrier.
      // Level l + 1's flag was last read at level l - 2, by every thread before
      // the barrier that ended level l - 1, and is set only after the barrier
      // that ends level l: level l clears it.
      for (int level = 1;; ++level) {
        if (tid == 0) sh_found[(level + 1) % 3] = 0;
        bool any = false;
        const uint32_t lv = (uint32_t)level * 0x01010101u;
        const double wlev = level <= 255 ? wl[level] : 0.0;
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
          const int v = tid + r * T;
          if (v >= n) continue;
          uint64_t acc[kWords] = {0, 0, 0, 0};
#pragma unroll
          for (int j = 0; j < kNbr; ++j)
            if (j < deg[r]) {
#pragma unroll
              for (int k = 0; k < kWords; ++k) acc[k] |= F[nb[r][j] * kWords + k];
            }
          if (in_lds) {
#pragma unroll 4
            for (int e = (int)(e0[r] - ebase) + kNbr; e < (int)(e0[r] - ebase) + deg[r]; ++e) {
              const int u = cols[e];
#pragma unroll
              for (int k = 0; k < kWords; ++k) acc[k] |= F[u * kWords + k];
            }
          } else {
            for (int64_t e = e0[r] + kNbr; e < e0[r] + deg[r]; ++e) {
              const int u = (int)(col_idx[e] - G.v_off);
#pragma unroll
              for (int k = 0; k < kWords; ++k) acc[k] |= F[u * kWords + k];
            }
          }
#pragma unroll
          for (int k = 0; k < kWords; ++k) {
            const uint64_t old = vis[v * kWords + k];
            const uint64_t nw = acc[k] & ~old;
            N[v * kWords + k] = nw;
            if (nw == 0) continue;
            any = true;
            if (level > 255) continue;
            vis[v * kWords + k] = old | nw;
            ws[r] += (double)__popcll(nw) * wlev;
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
              for (int m = 0; m < 4; ++m)
                byt[r][k][c][m] |= lv & byte_mask4((uint32_t)(nw >> (16 * c + 4 * m)) & 0xfu);
          }
        }
        if (any) sh_found[level % 3] = 1;
        __syncthreads();
        const int a = sh_found[level % 3];
        if (!a) break;
        if (level > 255) {
          err = 1;
          break;
        }
        uint64_t* tmp = F;
        F = N;
        N = tmp;
      }
      // the sweep's bytes of the thread's rows (chunks past n_pad are not the graph's)
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        const int v = tid + r * T;
        if (v >= n) continue;
#pragma unroll
        for (int k = 0; k < kWords; ++k)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int s0 = base + 64 * k + 16 * c;
            if (s0 >= G.n_pad) continue;
            *reinterpret_cast<uint4*>(dg + ((size_t)(v / kRowBlock) * ng + s0 / kColGroup) * kTileBytes +
                                      (size_t)(v % kRowBlock) * kColGroup) =
                make_uint4(byt[r][k][c][0], byt[r][k][c][1], byt[r][k][c][2], byt[r][k][c][3]);
          }
      }
      __syncthreads();
    }
    if (err && tid == 0) status[gid] = -4;
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int v = tid + r * T;
      if (v < G.n_pad) Wg[G.w_off + v] = v < n ? ws[r] : 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// Layout, one graph per workgroup.  Work units of the all-pairs passes are
// (row block rb, column slice s): wave w takes units w, w + NW, ...; lane l of
// a unit owns row i = 64 rb + l and reads x_j as an LDS broadcast.
// ---------------------------------------------------------------------------
template <int DIM, int T>
__global__ __launch_bounds__(T) void k_batch_layout(const BatchGraph* __restrict__ graphs,
                                                    const int32_t* __restrict__ order, int count,
                                                    int32_t* __restrict__ queue, const uint8_t* __restrict__ d,
                                                    const double* __restrict__ Wg, float* __restrict__ X,
                                                    BatchResult* __restrict__ res, BatchParams p) {
  using V = typename VecT<DIM>::T;
  constexpr int NW = T / 64;
  __shared__ V xs[3][kBatchMaxN];
  __shared__ V es[kBatchMaxN];
  __shared__ double Ws[kBatchMaxN];
  __shared__ double Fp[kBatchMaxPartial * DIM];
  __shared__ float2 lut[256];
  __shared__ double red[8][NW];
  __shared__ double red_tot[8];
  __shared__ float lut2[256];  // -2/d
  __shared__ int sh_q;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  fill_weight_table<false>(lut);
  for (int b = tid; b < 256; b += T) lut2[b] = b ? -2.f * (1.0f / (float)b) : 0.f;
  const bool sg = p.safeguard && p.omega_p != 0.0;
  for (;;) {
    __syncthreads();
    if (tid == 0) sh_q = atomicAdd(queue, 1);
    __syncthreads();
    const int q = sh_q;
    if (q >= count) break;
    const int gid = order[q];
    const BatchGraph G = graphs[gid];
    const int n = G.n, n_pad = G.n_pad, nrb = n_pad / kRowBlock, ng = n_pad / kColGroup;
    const int S = G.slices, gps = (ng + S - 1) / S, units = nrb * S;
    const uint8_t* __restrict__ dg = d + G.d_off;
    for (int i = tid; i < n_pad; i += T) {
      V x;
      if constexpr (DIM == 2) {
        x = make_float2(0.f, 0.f);
        if (i < n) x = make_float2(X[(G.v_off + i) * 2], X[(G.v_off + i) * 2 + 1]);
      } else {
        x = make_float4(0.f, 0.f, 0.f, 0.f);
        if (i < n) x = make_float4(X[(G.v_off + i) * 3], X[(G.v_off + i) * 3 + 1], X[(G.v_off + i) * 3 + 2], 0.f);
      }
      xs[0][i] = x;
      xs[1][i] = x;
      xs[2][i] = x;
      es[i] = V{};
      Ws[i] = (i < n) ? Wg[G.w_off + i] : 0.0;
    }
    __syncthreads();
    int cur = 0, it = 0, rejected = 0, converged = n <= 1 ? 1 : 0, status = 0;
    double resid = 0.0;
    bool have_force = false;  // Fp holds the force at X^k (left by the last iteration's fused pass)
    while (it < p.max_iter && !converged && n > 1) {
      // ---- force pass at X^k: F_i = sum_j w (d - r) u_ij
      for (int u = have_force ? units : wave; u < units; u += NW) {
        const int rb = u % nrb, s = u / nrb;
        const int g0 = s * gps, g1 = min(g0 + gps, ng);
        const int i = rb * kRowBlock + lane;
        const V xi = xs[cur][i];
        const uint4* __restrict__ tile = reinterpret_cast<const uint4*>(dg + (size_t)rb * ng * kTileBytes) + lane;
        double F0 = 0.0, F1 = 0.0, F2 = 0.0;
        for (int g = g0; g < g1; ++g) {
          const uint4 qd = tile[(size_t)g * 64];
          float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
          for (int k = 0; k < kColGroup; ++k) {
            const float2 wt = lut[byte_of(chunk_word(qd, k), k & 3)];
            const V pj = xs[cur][g * kColGroup + k];
            const float dx = xi.x - pj.x, dy = xi.y - pj.y;
            float r2 = fmaf(dx, dx, kTiny);
            r2 = fmaf(dy, dy, r2);
            float dz = 0.f;
            if constexpr (DIM == 3) {
              dz = xi.z - pj.z;
              r2 = fmaf(dz, dz, r2);
            }
            const float c = fmaf(wt.x, __builtin_amdgcn_rsqf(r2), -wt.y);
            a0 = fmaf(c, dx, a0);
            a1 = fmaf(c, dy, a1);
            if constexpr (DIM == 3) a2 = fmaf(c, dz, a2);
            // keep the scheduler from hoisting all 16 LDS reads (VGPR pressure)
            if ((k & 3) == 3) __builtin_amdgcn_sched_barrier(0);
          }
          F0 += (double)a0;
          F1 += (double)a1;
          if constexpr (DIM == 3) F2 += (double)a2;
        }
        double* fp = Fp + ((size_t)s * n_pad + i) * DIM;
        fp[0] = F0;
        fp[1] = F1;
        if constexpr (DIM == 3) fp[2] = F2;
      }
      __syncthreads();
      // ---- Jacobi update x^H = x + F / W and extrapolation (eq. 11)
      const int h = (cur + 1) % 3, t = (cur + 2) % 3;
      double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int i = tid; i < n; i += T) {
        double F[3] = {0.0, 0.0, 0.0};
        for (int s = 0; s < S; ++s)
#pragma unroll
          for (int c = 0; c < DIM; ++c) F[c] += Fp[((size_t)s * n_pad + i) * DIM + c];
        const V x = xs[cur][i];
        const double Wi = Ws[i];
        float xv[3] = {x.x, x.y, 0.f};
        if constexpr (DIM == 3) xv[2] = x.z;
        float xh[3] = {0.f, 0.f, 0.f}, xt[3] = {0.f, 0.f, 0.f};
        bool bad = false;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
          xh[c] = (Wi > 0.0) ? (float)((double)xv[c] + F[c] / Wi) : xv[c];
          const double dl = (double)xh[c] - (double)xv[c];
          xt[c] = (float)((double)xh[c] + p.omega_p * dl);
          v[0] += dl * dl;
          v[1] += (double)xh[c] * (double)xh[c];
          v[2 + c] += (double)xh[c];
          bad = bad || !isfinite(xh[c]) || !isfinite(xt[c]);
        }
        if constexpr (DIM == 2) {
          xs[h][i] = make_float2(xh[0], xh[1]);
          xs[t][i] = make_float2(xt[0], xt[1]);
          es[i] = make_float2(xt[0] - xh[0], xt[1] - xh[1]);
        } else {
          xs[h][i] = make_float4(xh[0], xh[1], xh[2], 0.f);
          xs[t][i] = make_float4(xt[0], xt[1], xt[2], 0.f);
          es[i] = make_float4(xt[0] - xh[0], xt[1] - xh[1], xt[2] - xh[2], 0.f);
        }
        if (bad) v[6] += 1.0;
      }
      block_sum_waves<8, NW>(v, red, red_tot);
      // ---- the force at X~ (the next iteration's, if X~ is kept) with the
      // safeguard's bounds summed over the upper triangle in the same pass.  The
      // force terms are those of the pass above, in the same order.  For j > i,
      // with t = x~_i - x~_j, e = e_i - e_j (e = x~ - x^H), c the force
      // coefficient and w = 1/d^2, the pair's share of f(X~) - f(X^H) is
      // -c m - kappa delta^2 with m = e.(2t - e), kappa = 1/(d r~) >= 0 and
      // delta^2 <= |e|^2, so with P = sum_i e_i . F_i(X~):
      //   U = -2P + sum c |e|^2  >=  f(X~) - f(X^H)  >=  -2P - sum w |e|^2 = L.
      // U <= 0 keeps X~ and L > 0 keeps X^H; otherwise a pass over the upper
      // triangle sums the difference itself:
      //   r^H = sqrt|r~^2 - m|, term = m (1/d^2 - (2/d) / (r~ + r^H)).
      double df = 0.0;
      bool take_t = true;
      if (sg) {
        __syncthreads();  // the update has read every force partial
        double accB = 0.0, accC = 0.0;
        for (int u = wave; u < units; u += NW) {
          const int rb = u % nrb, s = u / nrb;
          const int gdiag = rb * (kRowBlock / kColGroup), gfree = gdiag + kRowBlock / kColGroup;
          const int g0 = s * gps, g1 = min(g0 + gps, ng);
          const int i = rb * kRowBlock + lane;
          const V xi = xs[t][i], ei = es[i];
          const uint4* __restrict__ tile = reinterpret_cast<const uint4*>(dg + (size_t)rb * ng * kTileBytes) + lane;
          double F0 = 0.0, F1 = 0.0, F2 = 0.0;
          // MODE 0: left of the diagonal block (force only); 1: the diagonal
          // block (j <= i masked); 2: right of it
          auto run = [&](auto mode_tag, int ga, int gb) {
            constexpr int MODE = decltype(mode_tag)::value;
            for (int g = ga; g < gb; ++g) {
              const uint4 qd = tile[(size_t)g * 64];
              const int jrel = i - g * kColGroup;
              float a0 = 0.f, a1 = 0.f, a2 = 0.f, ab = 0.f, ac = 0.f;
#pragma unroll
              for (int k = 0; k < kColGroup; ++k) {
                const uint32_t b = byte_of(chunk_word(qd, k), k & 3);
                const float2 wt = lut[b];
                const V pj = xs[t][g * kColGroup + k];
                const float dx = xi.x - pj.x, dy = xi.y - pj.y;
                float r2 = fmaf(dx, dx, kTiny);
                r2 = fmaf(dy, dy, r2);
                float dz = 0.f;
                if constexpr (DIM == 3) {
                  dz = xi.z - pj.z;
                  r2 = fmaf(dz, dz, r2);
                }
                const float c = fmaf(wt.x, __builtin_amdgcn_rsqf(r2), -wt.y);
                a0 = fmaf(c, dx, a0);
                a1 = fmaf(c, dy, a1);
                if constexpr (DIM == 3) a2 = fmaf(c, dz, a2);
                if constexpr (MODE != 0) {
                  const V pe = es[g * kColGroup + k];
                  const float ex = ei.x - pe.x, ey = ei.y - pe.y;
                  float e2 = fmaf(ex, ex, ey * ey);
                  if constexpr (DIM == 3) {
                    const float ez = ei.z - pe.z;
                    e2 = fmaf(ez, ez, e2);
                  }
                  if constexpr (MODE == 1) {
                    if (k <= jrel) e2 = 0.f;
                  }
                  ab = fmaf(c, e2, ab);
                  ac = fmaf(wt.y, e2, ac);
                }
                if ((k & 3) == 3) __builtin_amdgcn_sched_barrier(0);
              }
              F0 += (double)a0;
              F1 += (double)a1;
              if constexpr (DIM == 3) F2 += (double)a2;
              if constexpr (MODE != 0) {
                accB += (double)ab;
                accC += (double)ac;
              }
            }
          };
          run(std::integral_constant<int, 0>{}, g0, min(g1, gdiag));
          run(std::integral_constant<int, 1>{}, max(g0, gdiag), min(g1, gfree));
          run(std::integral_constant<int, 2>{}, max(g0, gfree), g1);
          double* fp = Fp + ((size_t)s * n_pad + i) * DIM;
          fp[0] = F0;
          fp[1] = F1;
          if constexpr (DIM == 3) fp[2] = F2;
        }
        __syncthreads();  // every force partial at X~ is written
        double pe = 0.0;  // P = sum_i e_i . F_i(X~), the force summed over slices as the update does
        for (int i = tid; i < n; i += T) {
          double F[3] = {0.0, 0.0, 0.0};
          for (int s = 0; s < S; ++s)
#pragma unroll
            for (int c = 0; c < DIM; ++c) F[c] += Fp[((size_t)s * n_pad + i) * DIM + c];
          const V e = es[i];
          pe += (double)e.x * F[0] + (double)e.y * F[1];
          if constexpr (DIM == 3) pe += (double)e.z * F[2];
        }
        double vb[3] = {accB, accC, pe};
        block_sum_waves<3, NW>(vb, red, red_tot);
        const double bu = -2.0 * vb[2] + vb[0], bl = -2.0 * vb[2] - vb[1];
        if (bu <= 0.0) {
          take_t = true;
        } else if (bl > 0.0) {
          take_t = false;
        } else {  // the bounds leave the sign open: the difference itself
          double acc = 0.0;
          for (int u = wave; u < units; u += NW) {
            const int rb = u % nrb, s = u / nrb;
            const int gdiag = rb * (kRowBlock / kColGroup), gfree = gdiag + kRowBlock / kColGroup;
            const int g0 = s * gps, g1 = min(g0 + gps, ng);
            const int i = rb * kRowBlock + lane;
            const V xi = xs[t][i], ei = es[i];
            const uint4* __restrict__ tile = reinterpret_cast<const uint4*>(dg + (size_t)rb * ng * kTileBytes) + lane;
            auto run = [&](auto mode_tag, int ga, int gb) {
              constexpr int MODE = decltype(mode_tag)::value;
              for (int g = ga; g < gb; ++g) {
                const uint4 qd = tile[(size_t)g * 64];
                const int jrel = i - g * kColGroup;
                float a = 0.f;
#pragma unroll
                for (int k = 0; k < kColGroup; ++k) {
                  const uint32_t b = byte_of(chunk_word(qd, k), k & 3);
                  const float2 wt = lut[b];
                  const V pj = xs[t][g * kColGroup + k];
                  const V pe = es[g * kColGroup + k];
                  const float dx = xi.x - pj.x, dy = xi.y - pj.y;
                  float r2 = fmaf(dx, dx, kTiny);
                  r2 = fmaf(dy, dy, r2);
                  const float ex = ei.x - pe.x, ey = ei.y - pe.y;
                  float m = ex * fmaf(2.f, dx, -ex);
                  m = fmaf(ey, fmaf(2.f, dy, -ey), m);
                  if constexpr (DIM == 3) {
                    const float dz = xi.z - pj.z, ez = ei.z - pe.z;
                    r2 = fmaf(dz, dz, r2);
                    m = fmaf(ez, fmaf(2.f, dz, -ez), m);
                  }
                  const float rinv = __builtin_amdgcn_rsqf(r2);
                  const float rh = __builtin_amdgcn_sqrtf(fabsf(r2 - m));
                  const float sum = fmaf(r2, rinv, rh);
                  float term = m * fmaf(lut2[b], __builtin_amdgcn_rcpf(sum), wt.y);
                  if constexpr (MODE == 1) {
                    if (k <= jrel) term = 0.f;
                  }
                  a += term;
                  if ((k & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                }
                acc += (double)a;
              }
            };
            run(std::integral_constant<int, 1>{}, max(g0, gdiag), min(g1, gfree));
            run(std::integral_constant<int, 2>{}, max(g0, gfree), g1);
          }
          double vv[1] = {acc};
          block_sum_waves<1, NW>(vv, red, red_tot);
          df = vv[0];
          take_t = df <= 0.0;
        }
      }
      // ---- decision and termination test (every thread holds the same sums)
      if (__builtin_amdgcn_readfirstlane(v[6] > 0.0 ? 1 : 0)) {
        status = -5;
        break;
      }
      const double mean2 = (v[2] * v[2] + v[3] * v[3] + (DIM == 3 ? v[4] * v[4] : 0.0)) / (double)n;
      const double den2 = v[1] - mean2;
      const double r = v[0] > 0.0 ? sqrt(v[0]) / sqrt(den2 > 0.0 ? den2 : 0.0) : 0.0;
      have_force = false;
      if (p.omega_p == 0.0) {
        cur = h;
      } else if (p.safeguard) {
        const bool take = take_t;
        cur = take ? t : h;
        have_force = take;  // the fused pass took the force at X~
        if (!take) ++rejected;
      } else {
        cur = t;
      }
      ++it;
      resid = r;
      if (r <= p.tol) converged = 1;
      // every thread computed the same decision from the same block sums
      cur = __builtin_amdgcn_readfirstlane(cur);
      have_force = __builtin_amdgcn_readfirstlane(have_force ? 1 : 0) != 0;
      converged = __builtin_amdgcn_readfirstlane(converged);
      rejected = __builtin_amdgcn_readfirstlane(rejected);
    }
    for (int i = tid; i < n; i += T) {
      const V x = xs[cur][i];
      X[(G.v_off + i) * DIM] = x.x;
      X[(G.v_off + i) * DIM + 1] = x.y;
      if constexpr (DIM == 3) X[(G.v_off + i) * DIM + 2] = x.z;
    }
    if (tid == 0) {
      BatchResult br;
      br.iterations = it;
      br.converged = converged;
      br.rejected = rejected;
      br.status = status;
      br.residual = resid;
      br.stress = 0.0;
      res[gid] = br;
    }
  }
}

__global__ void k_batch_reset(int32_t* queue) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *queue = 0;
}

__global__ __launch_bounds__(256) void k_fill_zero(uint8_t* __restrict__ p, size_t bytes) {
  const size_t chunks = (bytes + 15) / 16;
  for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < chunks; c += (size_t)gridDim.x * 256) {
    if (c * 16 + 16 <= bytes) {
      reinterpret_cast<uint4*>(p)[c] = make_uint4(0u, 0u, 0u, 0u);
    } else {
      for (size_t b = c * 16; b < bytes; ++b) p[b] = 0;
    }
  }
}

}  // namespace

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  const size_t chunks = (bytes + 15) / 16;
  const unsigned blocks = (unsigned)std::min<size_t>((chunks + 255) / 256, 4096);
  k_fill_zero<<<blocks, 256, 0, s>>>(reinterpret_cast<uint8_t*>(p), bytes);
  return hipGetLastError();
}

bool batch_threads_supported(int threads) { return threads == 256 || threads == 512 || threads == 1024; }

hipError_t launch_batch_reset(int32_t* queue, hipStream_t s) {
  k_batch_reset<<<1, 64, 0, s>>>(queue);
  return hipGetLastError();
}

hipError_t launch_batch_distances(int threads, int blocks, const BatchGraph* graphs, const int32_t* order, int count,
                                  int32_t* queue, const int64_t* row_ptr, const int32_t* col_idx, uint8_t* d,
                                  double* W, int32_t* status, hipStream_t s) {
  if (threads == 1024)
    k_batch_distances<1024><<<blocks, 1024, 0, s>>>(graphs, order, count, queue, row_ptr, col_idx, d, W, status);
  else if (threads == 512)
    k_batch_distances<512><<<blocks, 512, 0, s>>>(graphs, order, count, queue, row_ptr, col_idx, d, W, status);
  else
    k_batch_distances<256><<<blocks, 256, 0, s>>>(graphs, order, count, queue, row_ptr, col_idx, d, W, status);
  return hipGetLastError();
}

hipError_t launch_batch_layout(int dim, int threads, int blocks, const BatchGraph* graphs, const int32_t* order,
                               int count, int32_t* queue, const uint8_t* d, const double* W, float* X,
                               BatchResult* res, const BatchParams& p, hipStream_t s) {
#define SL_BATCH_LAUNCH(DD, TT) \
  k_batch_layout<DD, TT><<<blocks, TT, 0, s>>>(graphs, order, count, queue, d, W, X, res, p)
  if (dim == 2) {
    if (threads == 1024) SL_BATCH_LAUNCH(2, 1024);
    else if (threads == 512) SL_BATCH_LAUNCH(2, 512);
    else SL_BATCH_LAUNCH(2, 256);
  } else {
    if (threads == 1024) SL_BATCH_LAUNCH(3, 1024);
    else if (threads == 512) SL_BATCH_LAUNCH(3, 512);
    else SL_BATCH_LAUNCH(3, 256);
  }
#undef SL_BATCH_LAUNCH
  return hipGetLastError();
}

}  // namespace sl
