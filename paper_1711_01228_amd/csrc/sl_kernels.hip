// HIP kernels of libsorlayout for gfx950 (CDNA4, wave64).
//
// Per iteration of Algorithm 2 (Wang & Wang 2012) the loop runs
//   k_force    all-pairs pass at X^k: F_i = sum_j w_ij (d_ij - r_ij) u_ij, the
//              residual of eq. 5 (Prop. 2.1: L^X X - L^W X), optionally with the
//              stress terms of eq. 1
//   k_update   Jacobi sweep of eq. 5, X^H = X^k + F / W, and the extrapolation
//              X~ = X^H + (omega - 1)(X^H - X^k) of eq. 11, plus block sums for
//              the termination test
//   k_sgdelta  f(X~) - f(X^H) over unordered pairs (Alg. 2, safeguard)
//   k_select   the safeguard decision of Alg. 2, the termination test and the
//              iteration counter, in one workgroup
// The distances and W_i, built once per graph, are in sl_apsp.hip.
//
// Every cross-thread sum is taken in a fixed order (per-lane sequences, fixed
// trees, fixed slice order), so results are bitwise repeatable run to run.
#include "sl_device.h"

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

namespace sl {

namespace {

// ---------------------------------------------------------------------------
// All-pairs force pass.  One wave per (row block, column slice): lane l owns
// row i = 64 rb + l, streams its 16-byte distance chunks tile by tile, and
// reads the positions x_j of the slice through the scalar cache (j is uniform
// across the wave).  Per pair, with (1/d, w = 1/d^2) from the LDS table:
//   c    = w d / r - w = (1/d)(1/r) - w
//   F_i += c (x_i - x_j)          [= w (d - r) u_ij]
//   s_i += (r / d - 1)^2          [= w (r - d)^2]            (STRESS only)
// Sixteen pairs are summed in float, then folded into double accumulators.
// Pairs with d = 0 (i = j, no path, padding) give c = 0.
// ---------------------------------------------------------------------------
// Weights of distance k of a chunk: (1/d, 1/d^2) and, for the stress terms, 1
// when a path exists.  Bytes look the table up; floats divide (rcp).
template <bool FD, bool STRESS>
__device__ __forceinline__ typename WeightEntry<STRESS>::T pair_weights(const typename DChunkT<FD>::T& q, int k,
                                                                       const typename WeightEntry<STRESS>::T* lut) {
  if constexpr (FD) {
    const float dv = fchunk_at(q, k);
    const float inv = dv > 0.f ? __builtin_amdgcn_rcpf(dv) : 0.f;
    if constexpr (STRESS) return make_float4(inv, inv * inv, dv > 0.f ? 1.f : 0.f, 0.f);
    else return make_float2(inv, inv * inv);
  } else {
    return lut[byte_of(chunk_word(q, k), k & 3)];
  }
}

template <int DIM, bool STRESS, bool FD>
__global__ __launch_bounds__(256) void k_force(const uint8_t* __restrict__ d, const float* __restrict__ df,
                                               const float* __restrict__ Xb, size_t stride,
                                               const DevState* __restrict__ st, double* __restrict__ fpart,
                                               double* __restrict__ spart, int nrb, int ng, int gps, int n_pad,
                                               int cond) {
  using V = typename VecT<DIM>::T;
  using E = typename WeightEntry<STRESS>::T;
  using C = typename DChunkT<FD>::T;
  __shared__ E lut[256];
  if (st->done || (cond && !st->need_force)) return;
  if constexpr (!FD) {
    fill_weight_table<STRESS>(lut);
    __syncthreads();
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int rb = blockIdx.x * 4 + wave;
  if (rb >= nrb) return;
  const int slice = blockIdx.y;
  const int g0 = slice * gps;
  const int g1 = min(g0 + gps, ng);
  const V* __restrict__ X = reinterpret_cast<const V*>(Xb + (size_t)st->cur * stride);
  const int i = rb * kRowBlock + lane;
  const V xi = X[i];
  double F0 = 0.0, F1 = 0.0, F2 = 0.0, Sd = 0.0;
  auto group = [&](int g, const C& q) {
    const V* __restrict__ xj = X + (size_t)g * kColGroup;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, as = 0.f;
#pragma unroll
    for (int k = 0; k < kColGroup; ++k) {
      const E wt = pair_weights<FD, STRESS>(q, k, lut);
      const V p = xj[k];
      const float dx = xi.x - p.x, dy = xi.y - p.y;
      float r2 = fmaf(dx, dx, kTiny);
      r2 = fmaf(dy, dy, r2);
      float dz = 0.f;
      if constexpr (DIM == 3) {
        dz = xi.z - p.z;
        r2 = fmaf(dz, dz, r2);
      }
      const float rinv = __builtin_amdgcn_rsqf(r2);
      const float c = fmaf(wt.x, rinv, -wt.y);
      a0 = fmaf(c, dx, a0);
      a1 = fmaf(c, dy, a1);
      if constexpr (DIM == 3) a2 = fmaf(c, dz, a2);
      if constexpr (STRESS) {
        const float t = fmaf(r2 * rinv, wt.x, -wt.z);
        as = fmaf(t, t, as);
      }
    }
    F0 += (double)a0;
    F1 += (double)a1;
    if constexpr (DIM == 3) F2 += (double)a2;
    if constexpr (STRESS) Sd += (double)as;
  };
  if (g0 < g1) {
    // two chunk registers in turn (past the end the last group is loaded again:
    // in bounds, unused)
    C qa = load_chunk<FD>(d, df, rb, ng, g0, lane);
    for (int g = g0; g < g1; g += 2) {
      const C qb = load_chunk<FD>(d, df, rb, ng, min(g + 1, g1 - 1), lane);
      group(g, qa);
      if (g + 1 >= g1) break;
      qa = load_chunk<FD>(d, df, rb, ng, min(g + 2, g1 - 1), lane);
      group(g + 1, qb);
    }
  }
  double* fp = fpart + (size_t)slice * DIM * n_pad + i;
  fp[0] = F0;
  fp[n_pad] = F1;
  if constexpr (DIM == 3) fp[2 * (size_t)n_pad] = F2;
  if constexpr (STRESS) spart[(size_t)slice * n_pad + i] = Sd;
}

// ---------------------------------------------------------------------------
// Jacobi update and extrapolation, one thread per vertex.
//   x^H = x + F / W   (W = 0: the vertex has no partner and stays)
//   x~  = x^H + omega_p (x^H - x)                                  (eq. 11)
// Block sums (double): ||x^H - x||^2, ||x^H||^2, sum x^H per axis, stress
// terms, count of non-finite values.
// ---------------------------------------------------------------------------
template <int DIM, bool STRESS>
__global__ __launch_bounds__(256) void k_update(LoopParams p, const double* __restrict__ fpart,
                                                const double* __restrict__ spart, const double* __restrict__ W,
                                                float* __restrict__ Xb, size_t stride, float* __restrict__ Eb,
                                                const DevState* __restrict__ st, double* __restrict__ red) {
  using V = typename VecT<DIM>::T;
  __shared__ double sh[7][256];
  if (st->done) return;
  const int cur = st->cur, h = (cur + 1) % 3, t = (cur + 2) % 3;
  const V* __restrict__ X = reinterpret_cast<const V*>(Xb + (size_t)cur * stride);
  V* __restrict__ XH = reinterpret_cast<V*>(Xb + (size_t)h * stride);
  V* __restrict__ XT = reinterpret_cast<V*>(Xb + (size_t)t * stride);
  const int i = blockIdx.x * 256 + threadIdx.x;
  // factor of this iteration (schedule) and of this vertex (per-vertex factors)
  const double wp = p.omega_sched ? p.omega_sched[st->iter] : p.omega_p;
  const bool extrapolate = p.enumerate || p.omega_vertex || wp != 0.0;
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  if (i < p.n) {
    const double wpi = p.omega_vertex ? (double)p.omega_vertex[i] - 1.0 : wp;
    double F[3] = {0.0, 0.0, 0.0};
    if (!p.exact_y) {
#pragma unroll
      for (int c = 0; c < DIM; ++c) F[c] = sum_strided(fpart + (size_t)c * p.n_pad + i, p.slices, (size_t)DIM * p.n_pad);
    }
    const V x = X[i];
    const double Wi = W[i];
    float xv[3] = {x.x, x.y, 0.f};
    if constexpr (DIM == 3) xv[2] = x.z;
    float xh[3] = {0.f, 0.f, 0.f}, xt[3] = {0.f, 0.f, 0.f};
    bool bad = false;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      if (p.exact_y)  // the solve starts at Y = X^k and never moves held vertices
        xh[c] = (float)p.exact_y[(size_t)c * p.n_pad + i];
      else
        xh[c] = (Wi > 0.0) ? (float)((double)xv[c] + F[c] / Wi) : xv[c];
      const double dl = (double)xh[c] - (double)xv[c];
      xt[c] = (float)((double)xh[c] + wpi * dl);
      v[0] += dl * dl;
      v[1] += (double)xh[c] * (double)xh[c];
      v[2 + c] = (double)xh[c];
      bad = bad || !isfinite(xh[c]) || !isfinite(xt[c]);
    }
    V* __restrict__ E = reinterpret_cast<V*>(Eb);
    if constexpr (DIM == 2) {
      XH[i] = make_float2(xh[0], xh[1]);
      if (p.enumerate) {
        E[i] = make_float2(xh[0] - xv[0], xh[1] - xv[1]);  // the step X^H - X^k
      } else if (extrapolate) {
        XT[i] = make_float2(xt[0], xt[1]);
        E[i] = make_float2(xt[0] - xh[0], xt[1] - xh[1]);
      }
    } else {
      XH[i] = make_float4(xh[0], xh[1], xh[2], 0.f);
      if (p.enumerate) {
        E[i] = make_float4(xh[0] - xv[0], xh[1] - xv[1], xh[2] - xv[2], 0.f);
      } else if (extrapolate) {
        XT[i] = make_float4(xt[0], xt[1], xt[2], 0.f);
        E[i] = make_float4(xt[0] - xh[0], xt[1] - xh[1], xt[2] - xh[2], 0.f);
      }
    }
    if constexpr (STRESS) {
      v[5] += sum_strided(spart + i, p.slices, (size_t)p.n_pad);
    }
    v[6] = bad ? 1.0 : 0.0;
  }
  block_sum<7>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 7; ++k) red[(size_t)blockIdx.x * 8 + k] = v[k];
    red[(size_t)blockIdx.x * 8 + 7] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Safeguard: f(X~) - f(X^H) = sum_{i<j} w (r~ - r^H)(r~ + r^H - 2 d).
// Near convergence r~ and r^H agree to many digits, so neither r~ - r^H nor
// r~^2 - r^H^2 is formed as a difference.  With the stored step
// e_i = x~_i - x^H_i, h = x^H_i - x^H_j and e = e_i - e_j:
//   r~^2 - r^H^2 = e . (2h + e) =: m,     r~^2 = r^H^2 + m,
//   r~ - r^H = m / (r~ + r^H),
// and the pair term is w (r~ - r^H)(r~ + r^H - 2d) = m (1/d)(1/d - 2/(r~ + r^H)).
// Work items cover the upper triangle in equal runs of column groups: item =
// (row block, first group, end group); in the diagonal block pairs with
// j <= i are masked.  One double per wave, summed later in item order.
// ---------------------------------------------------------------------------
template <int DIM, bool MASK, bool FD>
__device__ __forceinline__ float safeguard_group(const typename DChunkT<FD>::T& q, const float* lut,
                                                 typename VecT<DIM>::T hi, typename VecT<DIM>::T ei,
                                                 const typename VecT<DIM>::T* __restrict__ hj,
                                                 const typename VecT<DIM>::T* __restrict__ ej, int jrel) {
  using V = typename VecT<DIM>::T;
  float a = 0.f;
#pragma unroll
  for (int k = 0; k < kColGroup; ++k) {
    float inv;
    if constexpr (FD) {
      const float dv = fchunk_at(q, k);
      inv = dv > 0.f ? __builtin_amdgcn_rcpf(dv) : 0.f;
    } else {
      inv = lut[byte_of(chunk_word(q, k), k & 3)];
    }
    const V ph = hj[k], pe = ej[k];
    const float hx = hi.x - ph.x, hy = hi.y - ph.y;
    const float ex = ei.x - pe.x, ey = ei.y - pe.y;
    float rh2 = fmaf(hx, hx, kTiny);
    rh2 = fmaf(hy, hy, rh2);
    float m = ex * fmaf(2.f, hx, ex);
    m = fmaf(ey, fmaf(2.f, hy, ey), m);
    if constexpr (DIM == 3) {
      const float hz = hi.z - ph.z, ez = ei.z - pe.z;
      rh2 = fmaf(hz, hz, rh2);
      m = fmaf(ez, fmaf(2.f, hz, ez), m);
    }
    // |.|: rounding may leave rh2 + m a hair below zero when x~_i and x~_j coincide
    const float rt2 = fabsf(rh2 + m);
    const float sum = fmaf(rh2, __builtin_amdgcn_rsqf(rh2), rt2 * __builtin_amdgcn_rsqf(rt2));
    float mi = m * inv;
    if constexpr (MASK) {
      if (k <= jrel) mi = 0.f;  // column j = i - jrel + k is not right of the diagonal
    }
    a = fmaf(mi, fmaf(-2.f, __builtin_amdgcn_rcpf(sum), inv), a);
  }
  return a;
}

template <int DIM, bool FD>
__global__ __launch_bounds__(256) void k_sgdelta(const uint8_t* __restrict__ d, const float* __restrict__ df,
                                                 const float* __restrict__ Xb, size_t stride,
                                                 const float* __restrict__ Eb, const int4* __restrict__ items,
                                                 int nitems, const DevState* __restrict__ st,
                                                 double* __restrict__ sgpart, int ng, int gate) {
  using V = typename VecT<DIM>::T;
  __shared__ float lut[256];
  if (st->done || (gate && !st->need_exact)) return;
  if constexpr (!FD) {
    lut[threadIdx.x] = threadIdx.x ? 1.0f / (float)threadIdx.x : 0.f;
    __syncthreads();
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int item = blockIdx.x * 4 + wave;
  if (item >= nitems) return;
  const int4 it = items[item];
  const int rb = it.x, g0 = it.y, g1 = it.z;
  const int h = (st->cur + 1) % 3;
  const V* __restrict__ XH = reinterpret_cast<const V*>(Xb + (size_t)h * stride);
  const V* __restrict__ E = reinterpret_cast<const V*>(Eb);
  const int gdiag = rb * (kRowBlock / kColGroup);
  const int gfree = gdiag + kRowBlock / kColGroup;  // first group right of the diagonal block
  const int i = rb * kRowBlock + lane;
  const V hi = XH[i], ei = E[i];
  double acc = 0.0;
  int g = g0;
  for (; g < g1 && g < gfree; ++g) {
    const auto q = load_chunk<FD>(d, df, rb, ng, g, lane);
    // pair (i, j) with j = 16 g + k is kept iff j > i, i.e. k > i - 16 g
    acc += (double)safeguard_group<DIM, true, FD>(q, lut, hi, ei, XH + (size_t)g * kColGroup,
                                                  E + (size_t)g * kColGroup, i - g * kColGroup);
  }
  for (; g < g1; ++g) {
    const auto q = load_chunk<FD>(d, df, rb, ng, g, lane);
    acc += (double)safeguard_group<DIM, false, FD>(q, lut, hi, ei, XH + (size_t)g * kColGroup,
                                                   E + (size_t)g * kColGroup, 0);
  }
  acc = wave_sum(acc);
  if (lane == 0) sgpart[item] = acc;
}

// ---------------------------------------------------------------------------
// The force pass at X~ with the safeguard of the same iteration folded in
// (Alg. 2's safeguard and the next iteration's force pass need the same pair
// geometry).  Every ordered pair takes its force term at X~ exactly as in
// k_force (same order and precision), so that if X~ is accepted the next
// iteration uses these sums as they are; otherwise k_force runs again at X^H.
// The pairs j > i also add their share of f(X~) - f(X^H), with
//   t = x~_i - x~_j,  e = e_i - e_j (e = x~ - x^H),  r~^2 = t.t,
//   m = r~^2 - r^H^2 = e.(2t - e)  (no difference of nearly equal squares),
//   r^H = sqrt|r~^2 - m|,  s = r~ + r^H,
//   term = w (r~ - r^H)(r~ + r^H - 2d) = m (1/d^2 - (2/d) / s).
// r^H^2 is formed as r~^2 - m: exact unless r^H << r~, where its error is
// small against s.  An iteration that does not extrapolate (a scheduled factor
// of 1) takes the force at X^H alone.  One double per workgroup (slice-major).
// Slices run right to left, the heavier (mostly upper-triangle) ones first.
// ---------------------------------------------------------------------------
template <int DIM, bool FD, int MODE>  // MODE 0: force only; 1: diagonal block (mask j <= i); 2: j > i throughout
__device__ __forceinline__ void force_sg_group(const typename DChunkT<FD>::T& q, const float4* lut,
                                               const typename VecT<DIM>::T& xi, const typename VecT<DIM>::T& ei,
                                               const typename VecT<DIM>::T* __restrict__ xj,
                                               const typename VecT<DIM>::T* __restrict__ ej, int jrel, float& a0,
                                               float& a1, float& a2, float& as) {
  using V = typename VecT<DIM>::T;
#pragma unroll
  for (int k = 0; k < kColGroup; ++k) {
    float inv, w, l2 = 0.f;
    if constexpr (FD) {
      const float dv = fchunk_at(q, k);
      inv = dv > 0.f ? __builtin_amdgcn_rcpf(dv) : 0.f;
      w = inv * inv;
      if constexpr (MODE != 0) l2 = -2.f * inv;
    } else {
      const uint32_t b = byte_of(chunk_word(q, k), k & 3);
      if constexpr (MODE != 0) {
        const float4 e4 = lut[b];
        inv = e4.x;
        w = e4.y;
        l2 = e4.z;
      } else {
        const float2 e2 = *reinterpret_cast<const float2*>(&lut[b]);
        inv = e2.x;
        w = e2.y;
      }
    }
    const V p = xj[k];
    const float tx = xi.x - p.x, ty = xi.y - p.y;
    float r2 = fmaf(tx, tx, kTiny);
    r2 = fmaf(ty, ty, r2);
    float tz = 0.f;
    if constexpr (DIM == 3) {
      tz = xi.z - p.z;
      r2 = fmaf(tz, tz, r2);
    }
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float c = fmaf(inv, rinv, -w);
    a0 = fmaf(c, tx, a0);
    a1 = fmaf(c, ty, a1);
    if constexpr (DIM == 3) a2 = fmaf(c, tz, a2);
    if constexpr (MODE != 0) {
      const V pe = ej[k];
      const float ex = ei.x - pe.x, ey = ei.y - pe.y;
      float m = ex * fmaf(2.f, tx, -ex);
      m = fmaf(ey, fmaf(2.f, ty, -ey), m);
      if constexpr (DIM == 3) {
        const float ez = ei.z - pe.z;
        m = fmaf(ez, fmaf(2.f, tz, -ez), m);
      }
      const float rh = __builtin_amdgcn_sqrtf(fabsf(r2 - m));
      const float sum = fmaf(r2, rinv, rh);
      float term = m * fmaf(l2, __builtin_amdgcn_rcpf(sum), w);
      if constexpr (MODE == 1) {
        if (k <= jrel) term = 0.f;  // column j = i - jrel + k is not right of the diagonal
      }
      as += term;
    }
  }
}

template <int DIM, bool FD>
__global__ __launch_bounds__(256) void k_force_sg(const uint8_t* __restrict__ d, const float* __restrict__ df,
                                                  const float* __restrict__ Xb, size_t stride,
                                                  const float* __restrict__ Eb, const double* __restrict__ omega_sched,
                                                  double omega_p, int vertex_factors, const DevState* __restrict__ st,
                                                  double* __restrict__ fpart, double* __restrict__ sgpart, int nrb,
                                                  int ng, int gps, int n_pad) {
  using V = typename VecT<DIM>::T;
  using C = typename DChunkT<FD>::T;
  __shared__ float4 lut[256];  // (1/d, 1/d^2, -2/d, 0)
  if (st->done) return;
  if constexpr (!FD) {
    for (int b = threadIdx.x; b < 256; b += blockDim.x) {
      const float fb = (float)b;
      const float inv = b ? 1.0f / fb : 0.f;
      lut[b] = make_float4(inv, b ? 1.0f / (fb * fb) : 0.f, -2.f * inv, 0.f);
    }
    __syncthreads();
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int rb = blockIdx.x * 4 + wave;
  const int slice = gridDim.y - 1 - blockIdx.y;
  if (rb >= nrb) {  // no rows: take part in the workgroup's sum only
    __syncthreads();
    return;
  }
  const int g0 = slice * gps;
  const int g1 = min(g0 + gps, ng);
  const double wp = omega_sched ? omega_sched[st->iter] : omega_p;
  const bool sg = vertex_factors || wp != 0.0;
  const int cur = st->cur;
  const V* __restrict__ X = reinterpret_cast<const V*>(Xb + (size_t)(sg ? (cur + 2) % 3 : (cur + 1) % 3) * stride);
  const V* __restrict__ E = reinterpret_cast<const V*>(Eb);
  const int i = rb * kRowBlock + lane;
  const V xi = X[i];
  const V ei = sg ? E[i] : V{};
  // column groups left of the diagonal block take the force only
  const int gdiag = sg ? rb * (kRowBlock / kColGroup) : ng;
  const int gfree = gdiag + kRowBlock / kColGroup;
  double F0 = 0.0, F1 = 0.0, F2 = 0.0, S = 0.0;
  auto run = [&](auto mode_tag, int ga, int gb) {
    constexpr int MODE = decltype(mode_tag)::value;
    if (ga >= gb) return;
    auto group = [&](int g, const C& q) {
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, as = 0.f;
      force_sg_group<DIM, FD, MODE>(q, lut, xi, ei, X + (size_t)g * kColGroup, E + (size_t)g * kColGroup,
                                    i - g * kColGroup, a0, a1, a2, as);
      F0 += (double)a0;
      F1 += (double)a1;
      if constexpr (DIM == 3) F2 += (double)a2;
      if constexpr (MODE != 0) S += (double)as;
    };
    // two chunk registers in turn: the next group loads while this one computes
    // (past the end the last group is loaded again: in bounds, unused)
    C qa = load_chunk<FD>(d, df, rb, ng, ga, lane);
    for (int g = ga; g < gb; g += 2) {
      const C qb = load_chunk<FD>(d, df, rb, ng, min(g + 1, gb - 1), lane);
      group(g, qa);
      if (g + 1 >= gb) break;
      qa = load_chunk<FD>(d, df, rb, ng, min(g + 2, gb - 1), lane);
      group(g + 1, qb);
    }
  };
  run(std::integral_constant<int, 0>{}, g0, min(g1, gdiag));
  run(std::integral_constant<int, 1>{}, max(g0, gdiag), min(g1, gfree));
  run(std::integral_constant<int, 2>{}, max(g0, gfree), g1);
  double* fp = fpart + (size_t)slice * DIM * n_pad + i;
  fp[0] = F0;
  fp[n_pad] = F1;
  if constexpr (DIM == 3) fp[2 * (size_t)n_pad] = F2;
  // one double per workgroup: the waves' sums in wave order
  __shared__ double wsum[4];
  S = wave_sum(S);
  if (lane == 0) wsum[wave] = S;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 4 && blockIdx.x * 4 + w < nrb; ++w) t += wsum[w];
    sgpart[(size_t)slice * gridDim.x + blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// Enumerating strategy (Sec. 5.2): f(X^H + c D) - f(X^H) for the paper's
// factors c = 0.5, 1.0, ..., 9.0 at once, D = X^H - X^k the stored step.  Per
// pair, with h = x^H_i - x^H_j, s = D_i - D_j, a = h.s, b = s.s:
//   r_c^2 - r^H^2 = c (2a + c b) =: m_c, and the term is m_c (1/d)(1/d - 2/(r_c + r^H))
// as in the safeguard.  One double per candidate and work item.
// ---------------------------------------------------------------------------
template <int DIM, bool MASK>
__device__ __forceinline__ void enum_group(const uint4& q, const float* lut, typename VecT<DIM>::T hi,
                                           typename VecT<DIM>::T di, const typename VecT<DIM>::T* __restrict__ hj,
                                           const typename VecT<DIM>::T* __restrict__ dj, int jrel,
                                           float (&a)[kEnumCandidates]) {
  using V = typename VecT<DIM>::T;
#pragma unroll 2
  for (int k = 0; k < kColGroup; ++k) {
    const float inv = lut[byte_of(chunk_word(q, k), k & 3)];
    const V ph = hj[k], pd = dj[k];
    const float hx = hi.x - ph.x, hy = hi.y - ph.y;
    const float sx = di.x - pd.x, sy = di.y - pd.y;
    float rh2 = fmaf(hx, hx, kTiny);
    rh2 = fmaf(hy, hy, rh2);
    float aa = fmaf(hy, sy, hx * sx), bb = fmaf(sy, sy, sx * sx);
    if constexpr (DIM == 3) {
      const float hz = hi.z - ph.z, sz = di.z - pd.z;
      rh2 = fmaf(hz, hz, rh2);
      aa = fmaf(hz, sz, aa);
      bb = fmaf(sz, sz, bb);
    }
    const float rh = rh2 * __builtin_amdgcn_rsqf(rh2);
    float ik = inv;
    if constexpr (MASK) {
      if (k <= jrel) ik = 0.f;
    }
    const float a2 = 2.f * aa;
#pragma unroll
    for (int c = 0; c < kEnumCandidates; ++c) {
      const float wc = 0.5f * (float)(c + 1);
      const float m = wc * fmaf(wc, bb, a2);
      const float rt2 = fabsf(rh2 + m);
      const float sum = fmaf(rt2, __builtin_amdgcn_rsqf(rt2), rh);
      a[c] = fmaf(m * ik, fmaf(-2.f, __builtin_amdgcn_rcpf(sum), inv), a[c]);
    }
  }
}

template <int DIM>
__global__ __launch_bounds__(256) void k_sgdelta_enum(const uint8_t* __restrict__ d, const float* __restrict__ Xb,
                                                      size_t stride, const float* __restrict__ Eb,
                                                      const int4* __restrict__ items, int nitems,
                                                      const DevState* __restrict__ st, double* __restrict__ sgpart,
                                                      int ng) {
  using V = typename VecT<DIM>::T;
  __shared__ float lut[256];
  if (st->done) return;
  lut[threadIdx.x] = threadIdx.x ? 1.0f / (float)threadIdx.x : 0.f;
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int item = blockIdx.x * 4 + wave;
  if (item >= nitems) return;
  const int4 it = items[item];
  const int rb = it.x, g0 = it.y, g1 = it.z;
  const int h = (st->cur + 1) % 3;
  const V* __restrict__ XH = reinterpret_cast<const V*>(Xb + (size_t)h * stride);
  const V* __restrict__ Dl = reinterpret_cast<const V*>(Eb);
  const int gdiag = rb * (kRowBlock / kColGroup);
  const int gfree = gdiag + kRowBlock / kColGroup;
  const int i = rb * kRowBlock + lane;
  const V hi = XH[i], di = Dl[i];
  const uint4* __restrict__ tile = reinterpret_cast<const uint4*>(d + (size_t)rb * ng * kTileBytes) + lane;
  double acc[kEnumCandidates];
#pragma unroll
  for (int c = 0; c < kEnumCandidates; ++c) acc[c] = 0.0;
  for (int g = g0; g < g1; ++g) {
    const uint4 q = tile[(size_t)g * 64];
    float a[kEnumCandidates];
#pragma unroll
    for (int c = 0; c < kEnumCandidates; ++c) a[c] = 0.f;
    if (g < gfree)
      enum_group<DIM, true>(q, lut, hi, di, XH + (size_t)g * kColGroup, Dl + (size_t)g * kColGroup,
                            i - g * kColGroup, a);
    else
      enum_group<DIM, false>(q, lut, hi, di, XH + (size_t)g * kColGroup, Dl + (size_t)g * kColGroup, 0, a);
#pragma unroll
    for (int c = 0; c < kEnumCandidates; ++c) acc[c] += (double)a[c];
  }
#pragma unroll
  for (int c = 0; c < kEnumCandidates; ++c) {
    const double t = wave_sum(acc[c]);
    if (lane == 0) sgpart[(size_t)item * kEnumCandidates + c] = t;
  }
}

// X~ = X^H + c D for the factor the select picked (enumerating strategy).
// Idempotent, so replays of a finished chunk leave X unchanged.
template <int DIM>
__global__ __launch_bounds__(256) void k_apply_enum(const float* __restrict__ Eb, float* __restrict__ Xb, size_t stride,
                                                    const DevState* __restrict__ st, int n) {
  using V = typename VecT<DIM>::T;
  if (!st->enum_pending) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int t = st->cur, h = (t + 2) % 3;
  const double c = st->enum_c;
  const V xh = reinterpret_cast<const V*>(Xb + (size_t)h * stride)[i];
  const V dl = reinterpret_cast<const V*>(Eb)[i];
  V* XT = reinterpret_cast<V*>(Xb + (size_t)t * stride);
  if constexpr (DIM == 2) {
    XT[i] = make_float2((float)((double)xh.x + c * dl.x), (float)((double)xh.y + c * dl.y));
  } else {
    XT[i] = make_float4((float)((double)xh.x + c * dl.x), (float)((double)xh.y + c * dl.y),
                        (float)((double)xh.z + c * dl.z), 0.f);
  }
}

// ---------------------------------------------------------------------------
// Alg. 2's safeguard, the loop's end and the termination test, one workgroup.
// mode kSelectPlain: sgpart holds partial sums of f(X~) - f(X^H).
// mode kSelectBounds: sgpart holds (B, C) per item and edot partial sums of
//   P = sum_i e_i . F_i(X~): U = -2P + B >= f(X~) - f(X^H) >= -2P - C = L.  U <= 0
//   keeps X~, L > 0 keeps X^H; otherwise the iteration is left open (need_exact)
//   for the exact pass and a kSelectExact select.
// mode kSelectExact: only when need_exact is set; as kSelectPlain.
// ---------------------------------------------------------------------------
// Sum of x[b * step + off] over b < count: eight independent sums per thread
// (loads in flight), added in a fixed order; every thread's share.
__device__ __forceinline__ double strided_share(const double* __restrict__ x, int count, int step, int off) {
  double u[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < count; b += 256 * 8) {
    // all 8 loads issued before any is used (a skipped one leaves its register
    // unwritten and is masked out after)
    double t[8];
    bool on[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      on[q] = b + q * 256 < count;
      if (on[q]) t[q] = x[(size_t)(b + q * 256) * step + off];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) u[q] += on[q] ? t[q] : 0.0;
  }
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) t += u[q];
  return t;
}

// The bounds' sums over the pass's records: B and C from the (B, C) pairs of
// the nsg items, P from the nedot records, and D from the items' differences
// when dpart is given.  Each thread keeps 16 independent sums of each (items
// t + 256 (16 r + u)), so 16 loads of each kind are in flight at once; the
// partials are added in a fixed order.
__device__ __forceinline__ void bounds_shares(const double* __restrict__ sgpart, int nsg,
                                              const double* __restrict__ edot, int nedot,
                                              const double* __restrict__ dpart, double& B, double& C, double& P,
                                              double& D) {
  constexpr int U = 16;
  double b[U], c[U], q[U], e[U];
#pragma unroll
  for (int u = 0; u < U; ++u) b[u] = c[u] = q[u] = e[u] = 0.0;
  const double2* __restrict__ bc = reinterpret_cast<const double2*>(sgpart);
  const int count = nsg > nedot ? nsg : nedot;
  for (int base = threadIdx.x; base < count; base += 256 * U) {
    // every load of the round issued before any is used (a skipped one leaves
    // its register unwritten and is masked out after)
    double2 x[U];
    double y[U], z[U];
    bool on_s[U], on_e[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = base + u * 256;
      on_s[u] = k < nsg;
      on_e[u] = k < nedot;
      if (on_s[u]) x[u] = bc[k];
      if (on_e[u]) y[u] = edot[k];
      if (dpart && on_s[u]) z[u] = dpart[k];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      b[u] += on_s[u] ? x[u].x : 0.0;
      c[u] += on_s[u] ? x[u].y : 0.0;
      q[u] += on_e[u] ? y[u] : 0.0;
      if (dpart) e[u] += on_s[u] ? z[u] : 0.0;
    }
  }
  B = C = P = D = 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    B += b[u];
    C += c[u];
    P += q[u];
    D += e[u];
  }
}

__global__ __launch_bounds__(256) void k_select(LoopParams p, const double* __restrict__ red, int nred,
                                                const double* __restrict__ sgpart, int nsg,
                                                DevState* __restrict__ st, double* __restrict__ trace, int dim,
                                                int mode, const double* __restrict__ edot, int nedot) {
  __shared__ double sh[11][256];
  __shared__ double cand[kEnumCandidates];
  if (st->done) return;
  if (mode == kSelectExact && !st->need_exact) return;
  const int k = st->iter;
  const double wp = p.omega_sched ? p.omega_sched[k] : p.omega_p;
  const int ran_exact = st->exact_next;  // which variant of the unordered fused pass ran
  double v[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nred; b += 256) {
#pragma unroll
    for (int q = 0; q < 7; ++q) v[q] += red[(size_t)b * 8 + q];
  }
  const bool sg = !p.enumerate && p.safeguard && (wp != 0.0 || p.omega_vertex);
  const bool bounds = sg && mode == kSelectBounds;
  if (bounds) {
    // B, C, P, and the difference summed by the exact variant
    bounds_shares(sgpart, nsg, edot, nedot, ran_exact ? sgpart + 2 * (size_t)nsg : nullptr, v[7], v[8], v[9],
                  v[10]);
  } else if (sg) {
    v[7] = strided_share(sgpart, nsg, 1, 0);
  }
  if (p.enumerate) {
    // 14 threads per candidate, each with eight independent sums over every
    // 14th item (loads in flight); the partials are added in thread order
    constexpr int kPerCand = 256 / kEnumCandidates;
    __shared__ double cpart[kEnumCandidates][kPerCand];
    const int c = threadIdx.x / kPerCand, j = threadIdx.x % kPerCand;
    if (c < kEnumCandidates) {
      double u[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int b = j; b < nsg; b += kPerCand * 8) {
        double t[8];  // all 8 loads issued before any is used
        bool on[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          on[q] = b + q * kPerCand < nsg;
          if (on[q]) t[q] = sgpart[(size_t)(b + q * kPerCand) * kEnumCandidates + c];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) u[q] += on[q] ? t[q] : 0.0;
      }
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) t += u[q];
      cpart[c][j] = t;
    }
    __syncthreads();
    if (threadIdx.x < kEnumCandidates) {
      double t = 0.0;
      for (int q = 0; q < kPerCand; ++q) t += cpart[threadIdx.x][q];
      cand[threadIdx.x] = t;
    }
  }
  block_sum<11>(v, sh);
  if (threadIdx.x != 0) return;
  if (v[6] > 0.0) {  // a non-finite coordinate: keep the last finite iterate
    st->status = -5;
    st->done = 1;
    return;
  }
  const double nan = __builtin_nan("");
  double df = sg ? v[7] : 0.0, bu = nan, bl = nan;
  bool take = true;
  if (bounds) {
    bu = -2.0 * v[9] + v[7];
    bl = -2.0 * v[9] - v[8];
    st->bound_u = bu;
    st->bound_l = bl;
    const bool decisive = bu <= 0.0 || bl > 0.0;
    if (ran_exact) {  // the pass summed the difference and U = sum -c m itself (no L)
      df = v[10];
      take = df <= 0.0;
      bu = v[7];
      bl = nan;
      st->bound_u = bu;
      st->bound_l = bl;
      st->exact_next = bu <= 0.0 ? 0 : 1;  // back to the bounds alone once U would have decided
    } else if (decisive) {
      df = nan;  // the difference itself is not formed when the bounds decide
      take = bu <= 0.0;
    } else {  // sign open: the exact pass and the second select take the iteration
      st->need_force = 0;
      st->need_exact = 1;
      return;
    }
  } else if (mode == kSelectExact) {
    take = df <= 0.0;
    bu = st->bound_u;
    bl = st->bound_l;
    st->need_exact = 0;
    st->exact_next = 1;  // the next fused pass sums the difference in as well
  } else {
    take = df <= 0.0;
  }
  const double dsq = v[0], hsq = v[1];
  const double mean2 = (v[2] * v[2] + v[3] * v[3] + (dim == 3 ? v[4] * v[4] : 0.0)) / (double)p.n;
  const double den2 = hsq - mean2;
  const double res = dsq > 0.0 ? sqrt(dsq) / sqrt(den2 > 0.0 ? den2 : 0.0) : 0.0;
  const int cur = st->cur, h = (cur + 1) % 3, t = (cur + 2) % 3;
  double accepted;
  st->need_force = 0;
  double used = p.omega_vertex ? __builtin_nan("") : wp;
  st->enum_pending = 0;
  if (p.enumerate) {
    int best = -1;  // -1: c = 0, difference 0; ties keep the smaller factor
    double bv = 0.0;
    for (int c = 0; c < kEnumCandidates; ++c)
      if (cand[c] < bv) {
        bv = cand[c];
        best = c;
      }
    df = bv;
    used = 0.5 * (best + 1);
    if (best < 0) {
      used = 0.0;
      st->cur = h;
      accepted = 0.0;
      st->rejected += 1;
    } else {
      st->cur = t;
      st->enum_c = used;
      st->enum_pending = 1;
      accepted = 1.0;
    }
  } else if (wp == 0.0 && !p.omega_vertex) {
    st->cur = h;
    accepted = -1.0;
  } else if (p.safeguard) {
    st->cur = take ? t : h;
    accepted = take ? 1.0 : 0.0;
    if (!take) st->rejected += 1;
    if (!take && p.fuse) st->need_force = 1;  // the pass after this one computed the force at X~
  } else {
    st->cur = t;
    accepted = 1.0;
  }
  st->omega_used = used;
  st->prev = cur;
  st->iter = k + 1;
  st->residual = res;
  st->last_df = df;
  if (trace) {
    double* row = trace + (size_t)k * kTraceCols;
    row[0] = res;
    row[1] = accepted;
    row[2] = df;
    row[3] = used;
    row[4] = p.stress ? 0.5 * v[5] : nan;
    row[5] = bu;
    row[6] = bl;
  }
  if (res <= p.tol) {
    st->converged = 1;
    st->done = 1;
  }
  if (k + 1 >= st->max_iter) st->done = 1;
}

// Copy the placement after the latest iteration into xtrace[iter - 1].
__global__ __launch_bounds__(256) void k_record(const float* __restrict__ Xb, size_t stride,
                                                const DevState* __restrict__ st, float* __restrict__ xtrace, int n,
                                                int dim) {
  const int it = st->iter;
  if (it <= 0) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int vec = dim == 2 ? 2 : 4;
  const float* src = Xb + (size_t)st->cur * stride + (size_t)i * vec;
  float* dst = xtrace + ((size_t)(it - 1) * n + i) * dim;
  for (int c = 0; c < dim; ++c) dst[c] = src[c];
}

// f = (1/2) sum_i s_i over the stress partials of one force pass.
// f = half the sum of the stress terms: first each vertex's sum over the slices
// (into slice 0, which only that vertex's thread reads), then one block.
__global__ __launch_bounds__(256) void k_stress_rows(double* __restrict__ spart, int slices, int n_pad) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n_pad) spart[i] = sum_strided(spart + i, slices, (size_t)n_pad);
}

__global__ __launch_bounds__(256) void k_stress_sum(const double* __restrict__ spart, int n_pad,
                                                    DevState* __restrict__ st) {
  __shared__ double sh[1][256];
  const int per = (n_pad + 255) / 256;
  double v[1] = {threadIdx.x * per < n_pad ? sum_strided(spart + threadIdx.x * per,
                                                         min(per, n_pad - (int)threadIdx.x * per), 1) : 0.0};
  block_sum<1>(v, sh);
  if (threadIdx.x == 0) st->stress = 0.5 * v[0];
}

// Caller placement (n x dim, row-major) -> iterate buffer (float2/float4, padded
// with zeros up to n_pad).
__global__ __launch_bounds__(256) void k_pack_in(const float* __restrict__ X, float* __restrict__ Xb, int n,
                                                 int n_pad, int dim) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n_pad) return;
  const int vec = dim == 2 ? 2 : 4;
  for (int c = 0; c < vec; ++c) Xb[(size_t)i * vec + c] = (i < n && c < dim) ? X[(size_t)i * dim + c] : 0.f;
}

__global__ __launch_bounds__(256) void k_pack_out(const float* __restrict__ Xb, const DevState* __restrict__ st,
                                                  size_t stride, float* __restrict__ X, int n, int dim) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int vec = dim == 2 ? 2 : 4;
  const float* src = Xb + (size_t)st->cur * stride + (size_t)i * vec;
  for (int c = 0; c < dim; ++c) X[(size_t)i * dim + c] = src[c];
}

__global__ __launch_bounds__(256) void k_gather_rows(const uint8_t* __restrict__ d, const float* __restrict__ df,
                                                     const int32_t* __restrict__ rows, int nrows, int n, int ng,
                                                     float* __restrict__ out) {
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= (size_t)nrows * n) return;
  const int k = (int)(q / n), j = (int)(q % n);
  const size_t o = tile_offset(rows[k], j, ng);
  out[q] = df ? df[o] : (float)d[o];
}

inline unsigned blocks_for(size_t items) { return (unsigned)((items + 255) / 256); }

}  // namespace

Split make_split(int n_pad) {
  Split sp;
  sp.nrb = n_pad / kRowBlock;
  sp.ng = n_pad / kColGroup;
  // About 32 waves per SIMD over the chip (256 CUs x 4 SIMDs): four rounds of
  // 8 resident waves, so that the dispatcher can even out passes whose waves
  // differ in work (the fused safeguard's upper triangle); at least 8 column
  // groups (128 columns) per wave.
  const int max_slices = std::max(1, sp.ng / 8);
  const int want = std::max(1, 32768 / std::max(1, sp.nrb));
  int slices = std::min(max_slices, want);
  sp.groups_per_slice = (sp.ng + slices - 1) / slices;
  sp.slices = (sp.ng + sp.groups_per_slice - 1) / sp.groups_per_slice;
  sp.blocks_x = (sp.nrb + 3) / 4;
  return sp;
}

hipError_t launch_fill_u8(uint8_t* p, size_t bytes, hipStream_t s) { return hipMemsetAsync(p, 0, bytes, s); }

hipError_t launch_pack_in(const float* X, float* Xb, int n, int n_pad, int dim, hipStream_t s) {
  k_pack_in<<<blocks_for(n_pad), 256, 0, s>>>(X, Xb, n, n_pad, dim);
  return hipGetLastError();
}

hipError_t launch_pack_out(const float* Xb, const DevState* st, size_t stride, float* X, int n, int dim,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_pack_out<<<blocks_for(n), 256, 0, s>>>(Xb, st, stride, X, n, dim);
  return hipGetLastError();
}

template <int DIM, bool STRESS>
static void force_launch(const uint8_t* d, const float* df, const float* Xb, size_t stride, const DevState* st,
                         double* fpart, double* spart, const Split& sp, int n_pad, hipStream_t s, int cond = 0) {
  const dim3 grid(sp.blocks_x, sp.slices);
  if (df)
    k_force<DIM, STRESS, true><<<grid, 256, 0, s>>>(d, df, Xb, stride, st, fpart, spart, sp.nrb, sp.ng,
                                                     sp.groups_per_slice, n_pad, cond);
  else
    k_force<DIM, STRESS, false><<<grid, 256, 0, s>>>(d, df, Xb, stride, st, fpart, spart, sp.nrb, sp.ng,
                                                      sp.groups_per_slice, n_pad, cond);
}

hipError_t launch_force_cond(int dim, const uint8_t* d, const float* df, const float* Xb, size_t stride,
                             const DevState* st, double* fpart, const Split& sp, int n_pad, hipStream_t s) {
  if (dim == 2) force_launch<2, false>(d, df, Xb, stride, st, fpart, nullptr, sp, n_pad, s, 1);
  else force_launch<3, false>(d, df, Xb, stride, st, fpart, nullptr, sp, n_pad, s, 1);
  return hipGetLastError();
}

template <int DIM, bool FD>
static void force_sg_launch(const LoopParams& lp, const uint8_t* d, const float* df, const float* Xb, size_t stride,
                            const float* Eb, const DevState* st, double* fpart, double* sgpart, const Split& sp,
                            hipStream_t s) {
  const dim3 grid(sp.blocks_x, sp.slices);
  k_force_sg<DIM, FD><<<grid, 256, 0, s>>>(d, df, Xb, stride, Eb, lp.omega_sched, lp.omega_p,
                                            lp.omega_vertex ? 1 : 0, st, fpart, sgpart, sp.nrb, sp.ng,
                                            sp.groups_per_slice, lp.n_pad);
}

hipError_t launch_force_sg(int dim, const LoopParams& lp, const uint8_t* d, const float* df, const float* Xb,
                           size_t stride, const float* Eb, const DevState* st, double* fpart, double* sgpart,
                           const Split& sp, hipStream_t s) {
  if (dim == 2) {
    if (df) force_sg_launch<2, true>(lp, d, df, Xb, stride, Eb, st, fpart, sgpart, sp, s);
    else force_sg_launch<2, false>(lp, d, df, Xb, stride, Eb, st, fpart, sgpart, sp, s);
  } else {
    if (df) force_sg_launch<3, true>(lp, d, df, Xb, stride, Eb, st, fpart, sgpart, sp, s);
    else force_sg_launch<3, false>(lp, d, df, Xb, stride, Eb, st, fpart, sgpart, sp, s);
  }
  return hipGetLastError();
}

hipError_t launch_force(int dim, bool stress, const uint8_t* d, const float* df, const float* Xb, size_t stride,
                        const DevState* st, double* fpart, double* spart, const Split& sp, int n_pad,
                        hipStream_t s) {
  if (dim == 2) {
    if (stress) force_launch<2, true>(d, df, Xb, stride, st, fpart, spart, sp, n_pad, s);
    else force_launch<2, false>(d, df, Xb, stride, st, fpart, spart, sp, n_pad, s);
  } else {
    if (stress) force_launch<3, true>(d, df, Xb, stride, st, fpart, spart, sp, n_pad, s);
    else force_launch<3, false>(d, df, Xb, stride, st, fpart, spart, sp, n_pad, s);
  }
  return hipGetLastError();
}

hipError_t launch_update(int dim, const LoopParams& p, const double* fpart, const double* spart,
                         const double* W, float* Xb, size_t stride, float* Eb, const DevState* st, double* red,
                         hipStream_t s) {
  const unsigned nb = blocks_for(p.n_pad);
  if (dim == 2) {
    if (p.stress) k_update<2, true><<<nb, 256, 0, s>>>(p, fpart, spart, W, Xb, stride, Eb, st, red);
    else k_update<2, false><<<nb, 256, 0, s>>>(p, fpart, spart, W, Xb, stride, Eb, st, red);
  } else {
    if (p.stress) k_update<3, true><<<nb, 256, 0, s>>>(p, fpart, spart, W, Xb, stride, Eb, st, red);
    else k_update<3, false><<<nb, 256, 0, s>>>(p, fpart, spart, W, Xb, stride, Eb, st, red);
  }
  return hipGetLastError();
}

std::vector<int4> triangle_items(const Split& sp) {
  // equal runs of column groups over the upper triangle (block granularity)
  int64_t total = 0;
  for (int rb = 0; rb < sp.nrb; ++rb) total += sp.ng - rb * (kRowBlock / kColGroup);
  const int run = (int)std::max<int64_t>(8, (total + 8191) / 8192);
  std::vector<int4> items;
  for (int rb = 0; rb < sp.nrb; ++rb)
    for (int g0 = rb * (kRowBlock / kColGroup); g0 < sp.ng; g0 += run)
      items.push_back(make_int4(rb, g0, std::min(g0 + run, sp.ng), 0));
  return items;
}

hipError_t launch_sgdelta(int dim, const uint8_t* d, const float* df, const float* Xb, size_t stride,
                          const float* Eb, const int4* items, int nitems, const DevState* st, double* sgpart,
                          const Split& sp, hipStream_t s, int gate) {
  const unsigned nb = (unsigned)((nitems + 3) / 4);
  if (dim == 2) {
    if (df) k_sgdelta<2, true><<<nb, 256, 0, s>>>(d, df, Xb, stride, Eb, items, nitems, st, sgpart, sp.ng, gate);
    else k_sgdelta<2, false><<<nb, 256, 0, s>>>(d, df, Xb, stride, Eb, items, nitems, st, sgpart, sp.ng, gate);
  } else {
    if (df) k_sgdelta<3, true><<<nb, 256, 0, s>>>(d, df, Xb, stride, Eb, items, nitems, st, sgpart, sp.ng, gate);
    else k_sgdelta<3, false><<<nb, 256, 0, s>>>(d, df, Xb, stride, Eb, items, nitems, st, sgpart, sp.ng, gate);
  }
  return hipGetLastError();
}

hipError_t launch_sgdelta_enum(int dim, const uint8_t* d, const float* Xb, size_t stride, const float* Eb,
                               const int4* items, int nitems, const DevState* st, double* sgpart, const Split& sp,
                               hipStream_t s) {
  const unsigned nb = (unsigned)((nitems + 3) / 4);
  if (dim == 2) k_sgdelta_enum<2><<<nb, 256, 0, s>>>(d, Xb, stride, Eb, items, nitems, st, sgpart, sp.ng);
  else k_sgdelta_enum<3><<<nb, 256, 0, s>>>(d, Xb, stride, Eb, items, nitems, st, sgpart, sp.ng);
  return hipGetLastError();
}

hipError_t launch_apply_enum(const float* Eb, float* Xb, size_t stride, const DevState* st, int n, int dim,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (dim == 2) k_apply_enum<2><<<blocks_for(n), 256, 0, s>>>(Eb, Xb, stride, st, n);
  else k_apply_enum<3><<<blocks_for(n), 256, 0, s>>>(Eb, Xb, stride, st, n);
  return hipGetLastError();
}

hipError_t launch_select(int dim, const LoopParams& p, const double* red, int nred, const double* sgpart,
                         int nsg, DevState* st, double* trace, hipStream_t s, int mode, const double* edot,
                         int nedot) {
  k_select<<<1, 256, 0, s>>>(p, red, nred, sgpart, nsg, st, trace, dim, mode, edot, nedot);
  return hipGetLastError();
}

hipError_t launch_record(const float* Xb, size_t stride, const DevState* st, float* xtrace, int n, int dim,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_record<<<blocks_for(n), 256, 0, s>>>(Xb, stride, st, xtrace, n, dim);
  return hipGetLastError();
}

hipError_t launch_stress_sum(double* spart, int slices, int n_pad, DevState* st, hipStream_t s) {
  k_stress_rows<<<blocks_for(n_pad), 256, 0, s>>>(spart, slices, n_pad);
  k_stress_sum<<<1, 256, 0, s>>>(spart, n_pad, st);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const uint8_t* d, const float* df, const int32_t* rows, int nrows, int n, int ng,
                              float* out, hipStream_t s) {
  const size_t items = (size_t)nrows * n;
  if (items == 0) return hipSuccess;
  k_gather_rows<<<blocks_for(items), 256, 0, s>>>(d, df, rows, nrows, n, ng, out);
  return hipGetLastError();
}

}  // namespace sl
