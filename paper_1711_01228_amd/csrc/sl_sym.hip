// Force pass over unordered pairs (Newton's third law), on the vector units.
//
// F_i = sum_j c_ij (x_i - x_j) with c_ij = (1/d)(1/r) - 1/d^2 = c_ji, so each
// unordered pair i < j gives p = c_ij (x_i - x_j) to row i and -p to row j.
// Distances are hop-count bytes (weights from a table) or, for edge-length
// plans, floats (1/d by the reciprocal instruction, as the direct pass does).
// A work item (one wave) is a panel of 8 row strips (512 rows) and a run of up
// to 24 column groups right of the panel's diagonal block (shorter runs for
// small n, so that there are enough waves).  Per column group of 16
// columns the wave walks the strips (lane = row, the tile-major chunks of d as
// in the direct pass; pairs with j <= i masked where the group meets the
// diagonal):
//   rows     FP32 sum of p over the 16 columns, added into the strip's FP64
//            row sums (LDS, one slot per lane)
//   columns  per-lane FP32 sums of p over the 8 strips, then one
//            reduce-scatter across the wave (an exchange per lane bit), so that
//            lane 4 k holds the panel's total for column k of the group
// With SG the pass is taken at X~ (or at X^H for an iteration without
// extrapolation) and sums what bounds the safeguard of Alg. 2: with
// t = x~_i - x~_j, e = e_i - e_j (e = x~ - x^H as stored), c the pair's force
// coefficient at X~ and w = 1/d^2, each pair's share of f(X~) - f(X^H) is
//   w (r~ - r^H)(r~ + r^H - 2d) = -c m - kappa delta^2,
// m = r~^2 - r^H^2 = 2 e.t - |e|^2, kappa = 1/(d r~) >= 0, delta = r~ - r^H,
// and 0 <= delta^2 <= |e|^2 (triangle inequality).  So
//   U = sum -c m >= f(X~) - f(X^H) >= U - sum kappa |e|^2 = L,
// and since sum_{i<j} c (e_i - e_j).t = sum_i e_i . F_i(X~),
//   U = -2 P + B,  L = -2 P - C,  P = sum_i e_i . F_i,  B = sum c |e|^2,  C = sum w |e|^2.
// Per pair the pass adds B and C (every pair here has j > i); P comes from the
// reduction kernel, which has F_i.
// The column totals go out once per (panel, column) and the row sums once per
// (item, row), both as FP32; k_sym_reduce forms
//   F_i = sum over the items of i's panel of the row partials
//       - sum over the panels 0 .. panel(i) of the column partials
// in FP64 into force slice 0 (16 lanes per vertex, each over a fixed stride of
// the partials, then a fixed butterfly).  Every order is fixed, so results are
// bitwise repeatable.
#include "sl_device.h"

#include <algorithm>
#include <type_traits>

namespace sl {

namespace {

constexpr int kPanel = 8;   // row strips per work item (512 rows)
constexpr int kWaves = 4;   // work items (waves) per workgroup
constexpr int kChunk = 24;  // column groups per work item at most (measured: 20-24 best, 32 and up 8-10% slower)
constexpr int kMinItems = 8192;  // work items (waves) wanted at least: 8 per SIMD

typedef float vf16 __attribute__((ext_vector_type(16)));

// Reduce-scatter of the NR elements of R over the 64 lanes.  Each exchange
// step pairs the lanes that differ in one bit (5, 4, ...) and halves the
// elements; the lanes that still differ in the low bits then add their totals.
// Returns, in lane l, the total over all 64 lanes of element l >> (6 - log2 NR).
// (R is a vector value, not an array: the per-lane choice of element stays a
// register select.)
template <int NR, typename VF>
__device__ __forceinline__ float reduce_scatter(VF R, int lane) {
  constexpr int kSteps = NR == 16 ? 4 : 0;
  static_assert(kSteps > 0, "16 elements");
#pragma unroll
  for (int step = 0; step < kSteps; ++step) {
    const int bit = 5 - step;
    const int half = (NR / 2) >> step;
    const bool up = (lane >> bit) & 1;
#pragma unroll
    for (int r = 0; r < half; ++r) {
      const float lo = R[r], hi = R[r + half];
      const float send = up ? lo : hi;
      const float keep = up ? hi : lo;
      R[r] = keep + __shfl_xor(send, 1 << bit, 64);
    }
  }
  float t = R[0];
#pragma unroll
  for (int bit = 5 - kSteps; bit >= 0; --bit) t += __shfl_xor(t, 1 << bit, 64);
  return t;
}

// The same reduce-scatter for FP64 elements (the L^W matvec of the exact step).
typedef double vd16 __attribute__((ext_vector_type(16)));
__device__ __forceinline__ double reduce_scatter_d16(vd16 R, int lane) {
#pragma unroll
  for (int step = 0; step < 4; ++step) {
    const int bit = 5 - step;
    const int half = 8 >> step;
    const bool up = (lane >> bit) & 1;
#pragma unroll
    for (int r = 0; r < half; ++r) {
      const double lo = R[r], hi = R[r + half];
      const double send = up ? lo : hi;
      const double keep = up ? hi : lo;
      R[r] = keep + __shfl_xor(send, 1 << bit, 64);
    }
  }
  double t = R[0];
#pragma unroll
  for (int bit = 1; bit >= 0; --bit) t += __shfl_xor(t, 1 << bit, 64);
  return t;
}

// Gates of the pass (the state decides at run time which launches do work).
constexpr int kGateNone = 0;    // always
constexpr int kGateForce = 1;   // only when the force at X^H is still needed (after a rejection)
constexpr int kGateBounds = 2;  // only when the bounds alone are tried this iteration
constexpr int kGateExact = 3;   // only when the exact difference is summed in this iteration

__device__ __forceinline__ bool gate_closed(int gate, const DevState* st) {
  return st->done || (gate == kGateForce && !st->need_force) || (gate == kGateBounds && st->exact_next) ||
         (gate == kGateExact && !st->exact_next);
}

// -2/d of a weight-table entry (the entries of the exact variant carry it).
template <typename T>
__device__ __forceinline__ float lut_l2(const T& e) {
  if constexpr (std::is_same<T, float4>::value) return e.z;
  else return 0.f;
}

// SG = 0: force only.  SG = 1: the pass at X~ with the bounds' B and C.
// SG = 2: the pass at X~ with the exact f(X~) - f(X^H) summed in,
//   term = m (1/d^2 - (2/d) / s),  m = e.(2t - e),  s = r~ + r^H,
//   r^H = sqrt|r~^2 - m|  (no difference of nearly equal squares),
// and U = sum -c m pair by pair (its first B slot; C stays 0): whether the
// bounds alone would have decided the acceptance.
template <int DIM, int SG, bool FD>
__global__ __launch_bounds__(256) void k_force_sym(const uint8_t* __restrict__ d, const float* __restrict__ df,
                                                   const float* __restrict__ Xb,
                                                   size_t stride, const float* __restrict__ Eb,
                                                   const double* __restrict__ omega_sched, double omega_p,
                                                   int vertex_factors, int gate, const DevState* __restrict__ st,
                                                   const int4* __restrict__ items, int nitems,
                                                   float* __restrict__ Pi, float* __restrict__ Pj,
                                                   double* __restrict__ sgpart, int nb, int ng, int n_pad) {
  using V = typename VecT<DIM>::T;
  using L = std::conditional_t<SG == 2, float4, float2>;
  __shared__ L lut[256];                                  // (1/d, 1/d^2 [, -2/d, 0])
  __shared__ float rows[kWaves][kPanel][DIM][64];         // each wave's row sums of its 8 strips
  if (gate_closed(gate, st)) return;
  {
    const float fb = (float)threadIdx.x;
    const float inv = threadIdx.x ? 1.0f / fb : 0.f, w = threadIdx.x ? 1.0f / (fb * fb) : 0.f;
    if constexpr (SG == 2) lut[threadIdx.x] = make_float4(inv, w, -2.f * inv, 0.f);
    else lut[threadIdx.x] = make_float2(inv, w);
  }
  __syncthreads();  // the weight table; the waves are independent from here on
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int w_item = blockIdx.x * kWaves + wave;
  if (w_item >= nitems) return;
  const int4 it = items[w_item];
  const int panel = it.x, g0 = it.y, g1 = it.z, item = it.w;
  bool sg = false;
  int xbuf = st->cur;
  if constexpr (SG != 0) {
    const double wp = omega_sched ? omega_sched[st->iter] : omega_p;
    sg = vertex_factors || wp != 0.0;
    xbuf = sg ? (st->cur + 2) % 3 : (st->cur + 1) % 3;  // X~, or X^H without extrapolation
  }
  const V* __restrict__ X = reinterpret_cast<const V*>(Xb + (size_t)xbuf * stride);
  const V* __restrict__ E = reinterpret_cast<const V*>(Eb);
  const int nstrips = min(kPanel, nb - panel * kPanel);
  float (*racc)[DIM][64] = rows[wave];
  for (int r = 0; r < kPanel; ++r)
#pragma unroll
    for (int c = 0; c < DIM; ++c) racc[r][c][lane] = 0.f;
  double SB = 0.0, SC = 0.0, SD = 0.0;  // the item's B, C and exact difference

  for (int g = g0; g < g1; ++g) {
    const int jlo = g * kColGroup;
    const V* __restrict__ xj = X + jlo;
    const V* __restrict__ ej = E + jlo;
    // column sums of this group over the panel's rows (lane-wise partial sums)
    vf16 Cx = {}, Cy = {}, Cz = {};
    // strips 0 .. rfull - 1 lie wholly left of the group (every pair has j > i);
    // strips rfull .. rlast - 1 meet it on the diagonal (pairs with j <= i masked)
    const int rlast = min(nstrips, (jlo + kColGroup - 1) / 64 - panel * kPanel + 1);
    const int rfull = max(0, min(rlast, jlo / 64 - panel * kPanel));
    auto strips = [&](auto mask_tag, auto safe_tag, int ra, int rb) {
      constexpr bool MASK = decltype(mask_tag)::value;
      constexpr int SAFE = decltype(safe_tag)::value;  // 0, or SG
      if (ra >= rb) return;
      using C = typename DChunkT<FD>::T;
      C q = load_chunk<FD>(d, df, panel * kPanel + ra, ng, g, lane);
#pragma unroll 1
      for (int r = ra; r < rb; ++r) {
        const int ilo = (panel * kPanel + r) * 64;
        // the next strip's chunk loads while this one computes (the last strip loads itself again)
        const C qn = load_chunk<FD>(d, df, panel * kPanel + (r + 1 < rb ? r + 1 : r), ng, g, lane);
        const V xi = X[ilo + lane];
        V ei{};
        if constexpr (SAFE != 0) ei = E[ilo + lane];
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, ab = 0.f, ac = 0.f, ad = 0.f;
#pragma unroll
        for (int k = 0; k < kColGroup; ++k) {
          if constexpr (SAFE != 0 && DIM == 3) {
            // the columns' x_j and e_j are lane-uniform (scalar registers): 16 of
            // each in 3-D do not fit, so the second half loads after the first
            if (k % (kColGroup / 2) == 0) asm volatile("" ::: "memory");
          }
          float inv, w, l2 = 0.f;  // 1/d, 1/d^2, -2/d (0 where d = 0)
          if constexpr (FD) {
            const float dv = fchunk_at(q, k);
            inv = dv > 0.f ? __builtin_amdgcn_rcpf(dv) : 0.f;
            w = inv * inv;
            if constexpr (SAFE == 2) l2 = -2.f * inv;
          } else {
            const L e4 = lut[byte_of(chunk_word(q, k), k & 3)];
            inv = e4.x;
            w = e4.y;
            if constexpr (SAFE == 2) l2 = lut_l2(e4);
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
          float c = fmaf(inv, rinv, -w);
          if constexpr (MASK) {
            if (jlo + k <= ilo + lane) c = 0.f;
          }
          a0 = fmaf(c, tx, a0);
          a1 = fmaf(c, ty, a1);
          Cx[k] = fmaf(c, tx, Cx[k]);
          Cy[k] = fmaf(c, ty, Cy[k]);
          if constexpr (DIM == 3) {
            a2 = fmaf(c, tz, a2);
            Cz[k] = fmaf(c, tz, Cz[k]);
          }
          if constexpr (SAFE == 1) {  // B and C
            const V pe = ej[k];
            const float ex = ei.x - pe.x, ey = ei.y - pe.y;
            float e2 = fmaf(ex, ex, ey * ey);
            if constexpr (DIM == 3) {
              const float ez = ei.z - pe.z;
              e2 = fmaf(ez, ez, e2);
            }
            if constexpr (MASK) {
              if (jlo + k <= ilo + lane) e2 = 0.f;  // the pairs j <= i of a diagonal group
            }
            ab = fmaf(c, e2, ab);
            ac = fmaf(w, e2, ac);
          }
          if constexpr (SAFE == 2) {  // the difference itself, and U = sum -c m (c is 0 where masked)
            const V pe = ej[k];
            const float ex = ei.x - pe.x, ey = ei.y - pe.y;
            float m = ex * fmaf(2.f, tx, -ex);  // r~^2 - r^H^2 = e.(2t - e)
            m = fmaf(ey, fmaf(2.f, ty, -ey), m);
            if constexpr (DIM == 3) {
              const float ez = ei.z - pe.z;
              m = fmaf(ez, fmaf(2.f, tz, -ez), m);
            }
            const float rh = __builtin_amdgcn_sqrtf(fabsf(r2 - m));
            const float sum = fmaf(r2, rinv, rh);
            float term = m * fmaf(l2, __builtin_amdgcn_rcpf(sum), w);
            if constexpr (MASK) {
              if (jlo + k <= ilo + lane) term = 0.f;
            }
            ad += term;
            ab = fmaf(-c, m, ab);
          }
        }
        racc[r][0][lane] += a0;
        racc[r][1][lane] += a1;
        if constexpr (DIM == 3) racc[r][2][lane] += a2;
        if constexpr (SAFE != 0) {
          SB += (double)ab;
          SC += (double)ac;
        }
        if constexpr (SAFE == 2) SD += (double)ad;  // (SB holds U's partial here, SC stays 0)
        q = qn;
      }
    };
    if (sg) {
      strips(std::false_type{}, std::integral_constant<int, SG>{}, 0, rfull);
      strips(std::true_type{}, std::integral_constant<int, SG>{}, rfull, rlast);
    } else {
      strips(std::false_type{}, std::integral_constant<int, 0>{}, 0, rfull);
      strips(std::true_type{}, std::integral_constant<int, 0>{}, rfull, rlast);
    }
    // the group's column totals over the panel: lane l holds column l >> 2
    float* pj = Pj + ((size_t)panel * n_pad + jlo) * DIM;
    const float tx = reduce_scatter<16>(Cx, lane), ty = reduce_scatter<16>(Cy, lane);
    if ((lane & 3) == 0) {
      pj[(lane >> 2) * DIM] = tx;
      pj[(lane >> 2) * DIM + 1] = ty;
    }
    if constexpr (DIM == 3) {
      const float tz = reduce_scatter<16>(Cz, lane);
      if ((lane & 3) == 0) pj[(lane >> 2) * DIM + 2] = tz;
    }
  }
  for (int r = 0; r < nstrips; ++r) {
    float* out = Pi + ((size_t)item * kPanel * 64 + (size_t)r * 64 + lane) * DIM;
#pragma unroll
    for (int c = 0; c < DIM; ++c) out[c] = racc[r][c][lane];
  }
  if constexpr (SG != 0) {
    SB = wave_sum(SB);
    SC = wave_sum(SC);
    if (lane == 0) {
      sgpart[2 * (size_t)item] = SB;
      sgpart[2 * (size_t)item + 1] = SC;
    }
  }
  if constexpr (SG == 2) {
    SD = wave_sum(SD);
    if (lane == 0) sgpart[2 * (size_t)nitems + item] = SD;
  }
}

// 16 lanes per vertex: lane t of a vertex's group sums the row partials of
// items t, t + 16, ... and the column partials of panels t, t + 16, ... in
// FP64; the 16 sums are then added by a fixed butterfly, so every order is fixed.
constexpr int kReduceLanes = 16;

// With E (the fused pass), each workgroup also writes the sum of e_i . F_i over
// its 16 vertices into edot[block] (the P of the safeguard's bounds).
template <int DIM>
__global__ __launch_bounds__(256) void k_sym_reduce(const float* __restrict__ Pi, const float* __restrict__ Pj,
                                                    const int32_t* __restrict__ panel_items, int gate,
                                                    const DevState* __restrict__ st, double* __restrict__ fpart,
                                                    const float* __restrict__ Eb, double* __restrict__ edot,
                                                    int n_pad) {
  using V = typename VecT<DIM>::T;
  __shared__ double dots[256 / kReduceLanes];
  if (gate_closed(gate, st)) return;
  const int i = (blockIdx.x * 256 + threadIdx.x) / kReduceLanes;  // whole lane groups share i
  const int t = threadIdx.x % kReduceLanes;
  const bool live = i < n_pad;
  const int ii = live ? i : 0;
  const int strip = ii / 64, panel = strip / kPanel, row = ii % (kPanel * 64);
  double acc[DIM];
#pragma unroll
  for (int c = 0; c < DIM; ++c) acc[c] = 0.0;
  if (live) {
    for (int q = panel_items[panel] + t; q < panel_items[panel + 1]; q += kReduceLanes) {
      const float* p = Pi + ((size_t)q * kPanel * 64 + row) * DIM;
#pragma unroll
      for (int c = 0; c < DIM; ++c) acc[c] += (double)p[c];
    }
    for (int p = t; p <= panel; p += kReduceLanes) {
      const float* col = Pj + ((size_t)p * n_pad + ii) * DIM;
#pragma unroll
      for (int c = 0; c < DIM; ++c) acc[c] -= (double)col[c];
    }
  }
#pragma unroll
  for (int c = 0; c < DIM; ++c)
#pragma unroll
    for (int off = kReduceLanes / 2; off >= 1; off >>= 1) acc[c] += __shfl_xor(acc[c], off, 64);
  if (live && t == 0) {
#pragma unroll
    for (int c = 0; c < DIM; ++c) fpart[(size_t)c * n_pad + i] = acc[c];
  }
  if (Eb) {
    if (t == 0) {
      double dot = 0.0;
      if (live) {
        const V e = reinterpret_cast<const V*>(Eb)[i];
        dot = (double)e.x * acc[0] + (double)e.y * acc[1];
        if constexpr (DIM == 3) dot += (double)e.z * acc[2];
      }
      dots[threadIdx.x / kReduceLanes] = dot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int g = 0; g < 256 / kReduceLanes; ++g) s += dots[g];
      edot[blockIdx.x] = s;
    }
  }
}

// L^W p over unordered pairs, for the exact step's conjugate gradients (eq. 5):
// S_i = sum_{j != i} w_ij p_j with w = 1/d^2 = w_ji, so each unordered pair
// i < j gives w p_j to row i and w p_i to row j.  The work items, the strips and
// the tile-major chunks of d are those of the force pass; every product and sum
// is FP64 (an FP32 matvec stalls CG, see the exact step), the column totals of a
// group by the reduce-scatter, the row sums in LDS.  Row partials go out once
// per (item, row), column partials once per (panel, column), both FP64, and
// k_lw_sym_reduce forms q_i = W_i p_i - S_i.
template <int DIM>
__global__ __launch_bounds__(256) void k_lw_sym(const uint8_t* __restrict__ d, const double* __restrict__ pdb,
                                                const DevState* __restrict__ st, const CgState* __restrict__ cg,
                                                const int4* __restrict__ items, int nitems, double* __restrict__ Pi,
                                                double* __restrict__ Pj, int nb, int ng, int n_pad) {
  using P = std::conditional_t<DIM == 2, double2, double4>;
  __shared__ double lut[256];
  __shared__ double rows[kWaves][kPanel][DIM][64];  // each wave's FP64 row sums of its strips
  if (st->done || cg->done) return;
  lut[threadIdx.x] = threadIdx.x ? 1.0 / ((double)threadIdx.x * (double)threadIdx.x) : 0.0;
  __syncthreads();  // the weight table; the waves are independent from here on
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int w_item = blockIdx.x * kWaves + wave;
  if (w_item >= nitems) return;
  const int4 it = items[w_item];
  const int panel = it.x, g0 = it.y, g1 = it.z, item = it.w;
  const P* __restrict__ Pv = reinterpret_cast<const P*>(pdb);
  const int nstrips = min(kPanel, nb - panel * kPanel);
  double (*racc)[DIM][64] = rows[wave];
  for (int r = 0; r < kPanel; ++r)
#pragma unroll
    for (int c = 0; c < DIM; ++c) racc[r][c][lane] = 0.0;

  for (int g = g0; g < g1; ++g) {
    const int jlo = g * kColGroup;
    const P* __restrict__ pj = Pv + jlo;
    vd16 Cx = {}, Cy = {}, Cz = {};  // per-lane column sums of the group over the panel's strips
    const int rlast = min(nstrips, (jlo + kColGroup - 1) / 64 - panel * kPanel + 1);
    const int rfull = max(0, min(rlast, jlo / 64 - panel * kPanel));
    auto strips = [&](auto mask_tag, int ra, int rb) {
      constexpr bool MASK = decltype(mask_tag)::value;
      if (ra >= rb) return;
      uint4 q = load_chunk<false>(d, nullptr, panel * kPanel + ra, ng, g, lane);
#pragma unroll 1
      for (int r = ra; r < rb; ++r) {
        const int ilo = (panel * kPanel + r) * 64;
        // the next strip's chunk loads while this one computes
        const uint4 qn = load_chunk<false>(d, nullptr, panel * kPanel + (r + 1 < rb ? r + 1 : r), ng, g, lane);
        const P pi = Pv[ilo + lane];
        double q0 = 0.0, q1 = 0.0, q2 = 0.0;
        // the strip's 16 weights first: a table read issued among the scalar
        // loads of p_j waits for all of them (they share a counter and may
        // complete out of order)
        double wk[kColGroup];
#pragma unroll
        for (int k = 0; k < kColGroup; ++k) wk[k] = lut[byte_of(chunk_word(q, k), k & 3)];
#pragma unroll
        for (int k = 0; k < kColGroup; ++k) {
          // 16 columns' FP64 p_j (lane-uniform, scalar registers) do not fit at
          // once: each half (quarter in 3-D) loads after the previous one's work
          if (k % (DIM == 3 ? kColGroup / 4 : kColGroup / 2) == 0) asm volatile("" ::: "memory");
          double w = wk[k];
          if constexpr (MASK) {
            if (jlo + k <= ilo + lane) w = 0.0;  // the pairs j <= i of a diagonal group
          }
          const P pv = pj[k];
          q0 = fma(w, pv.x, q0);
          q1 = fma(w, pv.y, q1);
          Cx[k] = fma(w, pi.x, Cx[k]);
          Cy[k] = fma(w, pi.y, Cy[k]);
          if constexpr (DIM == 3) {
            q2 = fma(w, pv.z, q2);
            Cz[k] = fma(w, pi.z, Cz[k]);
          }
        }
        racc[r][0][lane] += q0;
        racc[r][1][lane] += q1;
        if constexpr (DIM == 3) racc[r][2][lane] += q2;
        q = qn;
      }
    };
    strips(std::false_type{}, 0, rfull);
    strips(std::true_type{}, rfull, rlast);
    // the group's column totals over the panel: lane l holds column l >> 2
    double* pjo = Pj + ((size_t)panel * n_pad + jlo) * DIM;
    const double tx = reduce_scatter_d16(Cx, lane), ty = reduce_scatter_d16(Cy, lane);
    if ((lane & 3) == 0) {
      pjo[(lane >> 2) * DIM] = tx;
      pjo[(lane >> 2) * DIM + 1] = ty;
    }
    if constexpr (DIM == 3) {
      const double tz = reduce_scatter_d16(Cz, lane);
      if ((lane & 3) == 0) pjo[(lane >> 2) * DIM + 2] = tz;
    }
  }
  for (int r = 0; r < nstrips; ++r) {
    double* out = Pi + ((size_t)item * kPanel * 64 + (size_t)r * 64 + lane) * DIM;
#pragma unroll
    for (int c = 0; c < DIM; ++c) out[c] = racc[r][c][lane];
  }
}

// q_i = W_i p_i - S_i, S_i = the row partials of the items of i's panel plus the
// column partials of panels 0 .. panel(i) (16 lanes per vertex, each over a
// fixed stride, then a fixed butterfly; a workgroup takes 64 vertices in four
// rounds), into slice 0 of qpart (column c at c n_pad), and the workgroup's
// record of sum_i p_i q_i per column.  The first workgroup also starts the
// step's counter (cg->ja = cg->jb), as the ordered matvec does.
constexpr int kLwReduceVertices = 64;
template <int DIM>
__global__ __launch_bounds__(256) void k_lw_sym_reduce(const double* __restrict__ Pi, const double* __restrict__ Pj,
                                                       const int32_t* __restrict__ panel_items,
                                                       const double* __restrict__ pdb, const double* __restrict__ W,
                                                       const DevState* __restrict__ st, CgState* __restrict__ cg,
                                                       double* __restrict__ qpart, double* __restrict__ pqrec,
                                                       int n_pad) {
  using P = std::conditional_t<DIM == 2, double2, double4>;
  __shared__ double sh[3][4];
  __shared__ double tot[3];
  if (st->done || cg->done) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) cg->ja = cg->jb;
  const int t = threadIdx.x % kReduceLanes, grp = threadIdx.x / kReduceLanes;
  double pq[3] = {0.0, 0.0, 0.0};
  for (int round = 0; round < kLwReduceVertices / (256 / kReduceLanes); ++round) {
    const int i = blockIdx.x * kLwReduceVertices + round * (256 / kReduceLanes) + grp;
    const bool live = i < n_pad;
    const int ii = live ? i : 0;
    const int strip = ii / 64, panel = strip / kPanel, row = ii % (kPanel * 64);
    double acc[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) acc[c] = 0.0;
    if (live) {
      for (int q = panel_items[panel] + t; q < panel_items[panel + 1]; q += kReduceLanes) {
        const double* p = Pi + ((size_t)q * kPanel * 64 + row) * DIM;
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[c] += p[c];
      }
      for (int p = t; p <= panel; p += kReduceLanes) {
        const double* col = Pj + ((size_t)p * n_pad + ii) * DIM;
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[c] += col[c];
      }
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
      for (int off = kReduceLanes / 2; off >= 1; off >>= 1) acc[c] += __shfl_xor(acc[c], off, 64);
    if (live && t == 0) {
      const P pv = reinterpret_cast<const P*>(pdb)[i];
      double pc[3] = {pv.x, pv.y, 0.0};
      if constexpr (DIM == 3) pc[2] = pv.z;
      const double Wi = W[i];
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        const double q = Wi * pc[c] - acc[c];
        qpart[(size_t)c * n_pad + i] = q;
        pq[c] += pc[c] * q;
      }
    }
  }
  block_sum_waves<3, 4>(pq, sh, tot);
  if (threadIdx.x == 0) {
    double* rec = pqrec + (size_t)blockIdx.x * 8;
#pragma unroll
    for (int k = 0; k < 3; ++k) rec[k] = pq[k];
    for (int k = 3; k < 8; ++k) rec[k] = 0.0;
  }
}

template <int DIM, int SG, bool FD>
void sym_launch(const LoopParams* lp, int gate, int reduce, const uint8_t* d, const float* df, const float* Xb,
                size_t stride, const float* Eb, const DevState* st, const int4* items, int nitems,
                const int32_t* panel_items, float* Pi, float* Pj, double* sgpart, double* fpart, double* edot,
                int n_pad, hipStream_t s) {
  const int nb = n_pad / 64, ng = n_pad / kColGroup;
  k_force_sym<DIM, SG, FD><<<(nitems + kWaves - 1) / kWaves, kWaves * 64, 0, s>>>(
      d, df, Xb, stride, Eb, lp ? lp->omega_sched : nullptr, lp ? lp->omega_p : 0.0, lp && lp->omega_vertex ? 1 : 0,
      gate, st, items, nitems, Pi, Pj, sgpart, nb, ng, n_pad);
  if (reduce == kSymReduceNone) return;
  k_sym_reduce<DIM><<<sym_reduce_blocks(n_pad), 256, 0, s>>>(Pi, Pj, panel_items,
                                                             reduce == kSymReduceAny ? kGateNone : gate, st, fpart,
                                                             SG != 0 ? Eb : nullptr, edot, n_pad);
}

template <int SG>
void sym_dispatch(int dim, const LoopParams* lp, int gate, int reduce, const uint8_t* d, const float* df,
                  const float* Xb, size_t stride, const float* Eb, const DevState* st, const int4* items, int nitems,
                  const int32_t* panel_items, float* Pi, float* Pj, double* sgpart, double* fpart, double* edot,
                  int n_pad, hipStream_t s) {
  if (dim == 2) {
    if (df) sym_launch<2, SG, true>(lp, gate, reduce, d, df, Xb, stride, Eb, st, items, nitems, panel_items, Pi, Pj,
                                    sgpart, fpart, edot, n_pad, s);
    else sym_launch<2, SG, false>(lp, gate, reduce, d, df, Xb, stride, Eb, st, items, nitems, panel_items, Pi, Pj,
                                  sgpart, fpart, edot, n_pad, s);
  } else {
    if (df) sym_launch<3, SG, true>(lp, gate, reduce, d, df, Xb, stride, Eb, st, items, nitems, panel_items, Pi, Pj,
                                    sgpart, fpart, edot, n_pad, s);
    else sym_launch<3, SG, false>(lp, gate, reduce, d, df, Xb, stride, Eb, st, items, nitems, panel_items, Pi, Pj,
                                  sgpart, fpart, edot, n_pad, s);
  }
}

}  // namespace

int sym_rows_per_item() { return kPanel * 64; }

unsigned sym_reduce_blocks(int n_pad) { return (unsigned)(((size_t)n_pad * kReduceLanes + 255) / 256); }

SymSplit make_sym_split(int n_pad) {
  SymSplit sp;
  sp.nb = n_pad / 64;
  sp.npanels = (sp.nb + kPanel - 1) / kPanel;
  const int ng = n_pad / kColGroup;
  // column groups right of each panel's diagonal block, over all panels; the
  // items shorten below kChunk groups until there are kMinItems of them
  long long groups = 0;
  for (int p = 0; p < sp.npanels; ++p) groups += ng - p * kPanel * (64 / kColGroup);
  const int chunk = (int)std::max<long long>(1, std::min<long long>(kChunk, groups / kMinItems));
  sp.panel_items.assign(sp.npanels + 1, 0);
  for (int p = 0; p < sp.npanels; ++p) {
    // the column groups right of the panel's first row: from its diagonal block on
    for (int g0 = p * kPanel * (64 / kColGroup); g0 < ng; g0 += chunk) {
      const int g1 = g0 + chunk < ng ? g0 + chunk : ng;
      sp.items.push_back(make_int4(p, g0, g1, (int)sp.items.size()));
    }
    sp.panel_items[p + 1] = (int)sp.items.size();
  }
  return sp;
}

hipError_t launch_force_sym(int dim, int cond, const uint8_t* d, const float* df, const float* Xb, size_t stride,
                            const DevState* st, const int4* items, int nitems, const int32_t* panel_items, float* Pi,
                            float* Pj, double* fpart, int n_pad, hipStream_t s) {
  sym_dispatch<0>(dim, nullptr, cond ? kGateForce : kGateNone, kSymReducePass, d, df, Xb, stride, nullptr, st, items,
                  nitems, panel_items, Pi, Pj, nullptr, fpart, nullptr, n_pad, s);
  return hipGetLastError();
}

unsigned lw_sym_reduce_blocks(int n_pad) { return (unsigned)((n_pad + kLwReduceVertices - 1) / kLwReduceVertices); }

hipError_t launch_lw_sym(int dim, const double* pd, const uint8_t* d, const double* W, const DevState* st, CgState* cg,
                         const LwSym& ls, double* qpart, double* pqrec, int n_pad, hipStream_t s) {
  const int nb = n_pad / 64, ng = n_pad / kColGroup;
  const unsigned blocks = (unsigned)((ls.nitems + kWaves - 1) / kWaves);
  if (dim == 2) {
    k_lw_sym<2><<<blocks, kWaves * 64, 0, s>>>(d, pd, st, cg, ls.items, ls.nitems, ls.Pi, ls.Pj, nb, ng, n_pad);
    k_lw_sym_reduce<2><<<lw_sym_reduce_blocks(n_pad), 256, 0, s>>>(ls.Pi, ls.Pj, ls.panel_items, pd, W, st, cg, qpart,
                                                                   pqrec, n_pad);
  } else {
    k_lw_sym<3><<<blocks, kWaves * 64, 0, s>>>(d, pd, st, cg, ls.items, ls.nitems, ls.Pi, ls.Pj, nb, ng, n_pad);
    k_lw_sym_reduce<3><<<lw_sym_reduce_blocks(n_pad), 256, 0, s>>>(ls.Pi, ls.Pj, ls.panel_items, pd, W, st, cg, qpart,
                                                                   pqrec, n_pad);
  }
  return hipGetLastError();
}

hipError_t launch_force_sym_sg(int dim, const LoopParams& lp, int exact, int gated, int reduce, const uint8_t* d,
                               const float* df, const float* Xb, size_t stride, const float* Eb, const DevState* st,
                               const int4* items, int nitems, const int32_t* panel_items, float* Pi, float* Pj,
                               double* sgpart, double* fpart, double* edot, int n_pad, hipStream_t s) {
  if (exact)
    sym_dispatch<2>(dim, &lp, gated ? kGateExact : kGateNone, reduce, d, df, Xb, stride, Eb, st, items, nitems,
                    panel_items, Pi, Pj, sgpart, fpart, edot, n_pad, s);
  else
    sym_dispatch<1>(dim, &lp, gated ? kGateBounds : kGateNone, reduce, d, df, Xb, stride, Eb, st, items, nitems,
                    panel_items, Pi, Pj, sgpart, fpart, edot, n_pad, s);
  return hipGetLastError();
}

}  // namespace sl
