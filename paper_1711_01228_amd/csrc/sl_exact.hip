// The exact step H of Algorithm 1/2 on the device: eq. 5, L^W X^H = L^X X^k,
// solved for every coordinate column by conjugate gradients with the diagonal
// of L^W (W_i) as preconditioner.
//
//   start      Y_0 = X^k, so r_0 = L^X X^k - L^W X^k = F, the force pass at X^k
//              (Prop. 2.1: the force on i is the residual of eq. 5)
//   step j     q = L^W p, (L^W p)_i = sum_j w_ij (p_i - p_j) = W_i p_i - sum_j w_ij p_j: an all-pairs pass
//              that streams one distance byte per ordered pair;
//              alpha = (r.z)/(p.q), Y += alpha p, r -= alpha q, z = r / W;
//              stop when ||r|| <= tol ||r_0|| (Frobenius over the columns) or
//              at the step limit, else beta = (r.z)_new/(r.z)_old, p = z + beta p
//   precision  the force pass (r_0) is FP32 per pair; the CG vectors and the
//              matvec are FP64: for smooth p the terms w (p_i - p_j) nearly
//              cancel, and an FP32 matvec stalls CG at about cond(L^W) * 1e-7
//   pinning    L^W is singular (one null vector per component) and eq. 5 fixes
//              X^H up to a translation of each component.  The lowest vertex of
//              each component keeps its place: its row and column are dropped
//              (r, z, p and q are held at 0 there), as the paper drops those of
//              x_1.  The reduced system is positive definite, so CG cannot
//              break down on the null-space part that FP32 rounding leaves in
//              F (its sum over a component is not exactly 0).
//
// CG vectors are double, structure of arrays (column c at c * n_pad); p is
// kept as double2/double4 per vertex, the layout the matvec reads.  Every grid-wide sum is a record
// of 8 doubles per 256-thread block, summed again by every block that needs it
// in the same fixed order, so all blocks take identical decisions and results
// are bitwise repeatable.
#include "sl_device.h"

#include <climits>

namespace sl {

namespace {

// Totals of fields first .. first+K-1 over nrec records of 8 doubles, summed in
// a fixed order; every thread of the 256-thread block receives them.
template <int K>
__device__ __forceinline__ void sum_records(const double* __restrict__ rec, int nrec, int first, double (&out)[K],
                                            double (*sh)[256]) {
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  for (int b = threadIdx.x; b < nrec; b += 256) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += rec[(size_t)b * 8 + first + k];
  }
  block_sum<K>(v, sh);  // ends with a barrier; sh[k][0] holds total k
#pragma unroll
  for (int k = 0; k < K; ++k) out[k] = sh[k][0];
  __syncthreads();
}

__device__ __forceinline__ const double* slot(const double* part, int s, int nblk) {
  return part + (size_t)s * nblk * 8;
}

// Lowest vertex of each vertex's component: min(i, min{j : d_ij > 0}).  A wave
// owns a row block and reads whole 1 KiB tiles; it stops once every lane has
// its answer (after the first tile on a connected graph).
__global__ __launch_bounds__(256) void k_components(const uint8_t* __restrict__ d, int32_t* __restrict__ comp, int n,
                                                    int ng) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int rb = i / kRowBlock, lane = i % kRowBlock;
  int best = (i < n) ? i : 0;
  const uint4* __restrict__ tile = reinterpret_cast<const uint4*>(d + (size_t)rb * ng * kTileBytes) + lane;
  for (int g = 0; g < ng; ++g) {
    if (__all(g * kColGroup >= best)) break;
    const uint4 q = tile[(size_t)g * 64];
    if (g * kColGroup < best) {
      for (int k = 0; k < kColGroup; ++k) {
        const int j = g * kColGroup + k;
        if (byte_of(chunk_word(q, k), k & 3) != 0u && j < best) {
          best = j;
          break;
        }
      }
    }
  }
  if (i < n) comp[i] = best;
}

template <int DIM> struct PVec;
template <> struct PVec<2> { using T = double2; };
template <> struct PVec<3> { using T = double4; };

template <int DIM>
__device__ __forceinline__ void store_p(double* pd, int i, const double (&pv)[3]) {
  using P = typename PVec<DIM>::T;
  if constexpr (DIM == 2) reinterpret_cast<P*>(pd)[i] = make_double2(pv[0], pv[1]);
  else reinterpret_cast<P*>(pd)[i] = make_double4(pv[0], pv[1], pv[2], 0.0);
}

// r_0 = F (force slices), Y = X^k, z = r / W, p = z; records slot 0 and the
// initial slot: [r.z per column, ||r||^2 per column].
template <int DIM>
__global__ __launch_bounds__(256) void k_cg_init(CgVectors v, const double* __restrict__ fpart, int slices,
                                                 const double* __restrict__ W, const int32_t* __restrict__ comp,
                                                 int n, const float* __restrict__ Xb, size_t stride,
                                                 const DevState* __restrict__ st, CgState* __restrict__ cg,
                                                 double* __restrict__ part, int nblk) {
  using V = typename VecT<DIM>::T;
  __shared__ double sh[6][256];
  if (st->done) return;
  const int n_pad = v.n_pad;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const V* __restrict__ X = reinterpret_cast<const V*>(Xb + (size_t)st->cur * stride);
  double acc[6] = {0, 0, 0, 0, 0, 0};
  if (i < n_pad) {
    const V x = X[i];
    float xv[3] = {x.x, x.y, 0.f};
    if constexpr (DIM == 3) xv[2] = x.z;
    const double Wi = W[i];
    const bool held = i >= n || comp[i] == i;  // dropped row (and padding)
    double pv[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const double r = held ? 0.0 : sum_strided(fpart + (size_t)c * n_pad + i, slices, (size_t)DIM * n_pad);
      const double z = Wi > 0.0 ? r / Wi : 0.0;
      const size_t o = (size_t)c * n_pad + i;
      v.y[o] = (double)xv[c];
      v.r[o] = r;
      v.z[o] = z;
      pv[c] = z;
      acc[c] = r * z;
      acc[3 + c] = r * r;
    }
    store_p<DIM>(v.pd, i, pv);
  }
  block_sum<6>(acc, sh);
  if (threadIdx.x == 0) {
    double* r0 = part + (size_t)blockIdx.x * 8;
    double* ri = part + ((size_t)kCgInitial * nblk + blockIdx.x) * 8;
#pragma unroll
    for (int k = 0; k < 6; ++k) r0[k] = ri[k] = acc[k];
    r0[6] = r0[7] = ri[6] = ri[7] = 0.0;
    if (blockIdx.x == 0) {
      cg->ja = 0;
      cg->jb = 0;
      cg->done = 0;
      cg->iters = 0;
      cg->rel = 1.0;
    }
  }
}

// q slices = L^W p over all ordered pairs, in the tiling of the force pass:
// one wave per (row block, column slice), p_j (double) through the scalar
// cache, w = 1/d^2 (double) from an LDS table, products and sums in double.
// (L^W p)_i = W_i p_i - sum_j w_ij p_j, with W_i the double row sum of the same
// weights: the pairs take one FMA per column, the slices -sum_j w_ij p_j, and
// slice 0 also W_i p_i.  For smooth p, where the terms w (p_i - p_j) nearly
// cancel, the one subtraction is done in double.  Each block also writes a
// record of sum_i p_i q_i(slice) per column (q is linear in the slices).
template <int DIM>
__global__ __launch_bounds__(256) void k_lw(const uint8_t* __restrict__ d, const double* __restrict__ pdb,
                                            const double* __restrict__ W,
                                            const DevState* __restrict__ st, CgState* __restrict__ cg,
                                            double* __restrict__ qpart, double* __restrict__ pqrec, int nrb, int ng,
                                            int gps, int n_pad) {
  using P = typename PVec<DIM>::T;
  __shared__ double lut[256];
  __shared__ double sh[3][4];
  __shared__ double tot[3];
  if (st->done || cg->done) return;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) cg->ja = cg->jb;
  lut[threadIdx.x] = threadIdx.x ? 1.0 / ((double)threadIdx.x * (double)threadIdx.x) : 0.0;
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int rb = blockIdx.x * 4 + wave;
  const int slice = blockIdx.y;
  double Q0 = 0.0, Q1 = 0.0, Q2 = 0.0;
  P pi{};
  if (rb < nrb) {
    const int g0 = slice * gps;
    const int g1 = min(g0 + gps, ng);
    const P* __restrict__ Pv = reinterpret_cast<const P*>(pdb);
    const int i = rb * kRowBlock + lane;
    pi = Pv[i];
    const uint4* __restrict__ tile = reinterpret_cast<const uint4*>(d + (size_t)rb * ng * kTileBytes) + lane;
    if (g0 < g1) {
      uint4 q = tile[(size_t)g0 * 64];
      for (int g = g0; g < g1; ++g) {
        uint4 qn = make_uint4(0u, 0u, 0u, 0u);
        if (g + 1 < g1) qn = tile[(size_t)(g + 1) * 64];
        const P* __restrict__ pj = Pv + (size_t)g * kColGroup;
        // the group's 16 weights first: a table read issued among the scalar
        // loads of p_j waits for all of them (they share a counter and may
        // complete out of order)
        double wk[kColGroup];
#pragma unroll
        for (int k = 0; k < kColGroup; ++k) wk[k] = lut[byte_of(chunk_word(q, k), k & 3)];
#pragma unroll
        for (int k = 0; k < kColGroup; ++k) {
          const double w = wk[k];
          const P pp = pj[k];
          Q0 = fma(w, pp.x, Q0);
          Q1 = fma(w, pp.y, Q1);
          if constexpr (DIM == 3) Q2 = fma(w, pp.z, Q2);
        }
        q = qn;
      }
    }
    const double Wi = slice == 0 ? W[i] : 0.0;
    Q0 = Wi * pi.x - Q0;
    Q1 = Wi * pi.y - Q1;
    if constexpr (DIM == 3) Q2 = Wi * pi.z - Q2;
    double* qp = qpart + (size_t)slice * DIM * n_pad + i;
    qp[0] = Q0;
    qp[n_pad] = Q1;
    if constexpr (DIM == 3) qp[2 * (size_t)n_pad] = Q2;
  }
  double pq[3] = {pi.x * Q0, pi.y * Q1, 0.0};
  if constexpr (DIM == 3) pq[2] = pi.z * Q2;
  block_sum_waves<3, 4>(pq, sh, tot);
  if (threadIdx.x == 0) {
    double* rec = pqrec + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 8;
#pragma unroll
    for (int k = 0; k < 3; ++k) rec[k] = pq[k];
    for (int k = 3; k < 8; ++k) rec[k] = 0.0;
  }
}

// alpha = (r.z)/(p.q) per column; Y += alpha p; r -= alpha q; z = r / W;
// record slot (j+1) % 2: [r.z, ||r||^2] per column.
template <int DIM>
__global__ __launch_bounds__(256) void k_cg_update(CgVectors v, const double* __restrict__ W,
                                                   const int32_t* __restrict__ comp, int n,
                                                   const double* __restrict__ qpart, int slices,
                                                   const DevState* __restrict__ st, const CgState* __restrict__ cg,
                                                   double* __restrict__ part, int nblk, const double* __restrict__ pqrec,
                                                   int npq) {
  __shared__ double sh[6][256];
  if (st->done || cg->done) return;
  const int j = cg->ja;
  const int n_pad = v.n_pad;
  double rz[3], pq[3], alpha[3];
  sum_records<3>(slot(part, j % 2, nblk), nblk, 0, rz, sh);
  sum_records<3>(pqrec, npq, 0, pq, sh);
#pragma unroll
  for (int c = 0; c < 3; ++c) alpha[c] = pq[c] > 0.0 ? rz[c] / pq[c] : 0.0;
  const int i = blockIdx.x * 256 + threadIdx.x;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  if (i < n_pad) {
    const double Wi = W[i];
    const bool held = i >= n || comp[i] == i;
    const typename PVec<DIM>::T pp = reinterpret_cast<const typename PVec<DIM>::T*>(v.pd)[i];
    double pv[3] = {pp.x, pp.y, 0.0};
    if constexpr (DIM == 3) pv[2] = pp.z;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const size_t o = (size_t)c * n_pad + i;
      const double q = held ? 0.0 : sum_strided(qpart + (size_t)c * n_pad + i, slices, (size_t)DIM * n_pad);
      v.y[o] += alpha[c] * pv[c];
      const double r = v.r[o] - alpha[c] * q;
      const double z = Wi > 0.0 ? r / Wi : 0.0;
      v.r[o] = r;
      v.z[o] = z;
      acc[c] = r * z;
      acc[3 + c] = r * r;
    }
  }
  block_sum<6>(acc, sh);
  if (threadIdx.x == 0) {
    double* rec = part + ((size_t)((j + 1) % 2) * nblk + blockIdx.x) * 8;
#pragma unroll
    for (int k = 0; k < 6; ++k) rec[k] = acc[k];
    rec[6] = rec[7] = 0.0;
  }
}

// Stop test ||r_{j+1}|| <= tol ||r_0|| or j + 1 = step limit; otherwise
// beta = (r.z)_{j+1} / (r.z)_j per column and p = z + beta p.
template <int DIM>
__global__ __launch_bounds__(256) void k_cg_dir(CgVectors v, const DevState* __restrict__ st,
                                                CgState* __restrict__ cg, const double* __restrict__ part, int nblk,
                                                double tol2, int max_steps) {
  __shared__ double sh[3][256];
  if (st->done || cg->done) return;
  const int j = cg->ja;
  const int n_pad = v.n_pad;
  double rzn[3], rrn[3], rzo[3], rr0[3];
  sum_records<3>(slot(part, (j + 1) % 2, nblk), nblk, 0, rzn, sh);
  sum_records<3>(slot(part, (j + 1) % 2, nblk), nblk, 3, rrn, sh);
  sum_records<3>(slot(part, j % 2, nblk), nblk, 0, rzo, sh);
  sum_records<3>(slot(part, kCgInitial, nblk), nblk, 3, rr0, sh);
  const double a = rrn[0] + rrn[1] + rrn[2], b = rr0[0] + rr0[1] + rr0[2];
  if (a <= tol2 * b || j + 1 >= max_steps) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      cg->done = 1;
      cg->iters = j + 1;
      cg->rel = b > 0.0 ? sqrt(a / b) : 0.0;
    }
    return;
  }
  double beta[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) beta[c] = rzo[c] > 0.0 ? rzn[c] / rzo[c] : 0.0;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n_pad) {
    using P = typename PVec<DIM>::T;
    const P po = reinterpret_cast<const P*>(v.pd)[i];
    double pold[3] = {po.x, po.y, 0.0};
    if constexpr (DIM == 3) pold[2] = po.z;
    double pv[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < DIM; ++c) pv[c] = v.z[(size_t)c * n_pad + i] + beta[c] * pold[c];
    store_p<DIM>(v.pd, i, pv);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) cg->jb = j + 1;
}

inline unsigned blocks_for(size_t items) { return (unsigned)((items + 255) / 256); }

}  // namespace

hipError_t launch_components(const uint8_t* d, int32_t* comp, int n, int n_pad, int ng, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_components<<<blocks_for(n_pad), 256, 0, s>>>(d, comp, n, ng);
  return hipGetLastError();
}

hipError_t launch_cg_init(int dim, const CgVectors& v, const double* fpart, int slices, const double* W,
                          const int32_t* comp, int n, const float* Xb, size_t stride, const DevState* st, CgState* cg,
                          double* part, hipStream_t s) {
  const int nblk = cg_blocks(v.n_pad);
  if (dim == 2) k_cg_init<2><<<nblk, 256, 0, s>>>(v, fpart, slices, W, comp, n, Xb, stride, st, cg, part, nblk);
  else k_cg_init<3><<<nblk, 256, 0, s>>>(v, fpart, slices, W, comp, n, Xb, stride, st, cg, part, nblk);
  return hipGetLastError();
}

hipError_t launch_lw(int dim, const CgVectors& v, const uint8_t* d, const double* W, const DevState* st, CgState* cg,
                     double* qpart, double* pqrec, const Split& sp, hipStream_t s) {
  const dim3 grid(sp.blocks_x, sp.slices);
  if (dim == 2)
    k_lw<2><<<grid, 256, 0, s>>>(d, v.pd, W, st, cg, qpart, pqrec, sp.nrb, sp.ng, sp.groups_per_slice, v.n_pad);
  else
    k_lw<3><<<grid, 256, 0, s>>>(d, v.pd, W, st, cg, qpart, pqrec, sp.nrb, sp.ng, sp.groups_per_slice, v.n_pad);
  return hipGetLastError();
}

hipError_t launch_cg_step(int dim, const CgVectors& v, const uint8_t* d, const double* W, const int32_t* comp, int n,
                          const DevState* st, CgState* cg, double* part, double* qpart, const Split& sp, double tol,
                          int max_steps, const LwSym* sym, hipStream_t s) {
  const int nblk = cg_blocks(v.n_pad);
  double* pqrec = part + (size_t)kCgSlots * nblk * 8;
  const int npq = sym ? (int)lw_sym_reduce_blocks(v.n_pad) : sp.blocks_x * sp.slices;
  const int slices = sym ? 1 : sp.slices;
  hipError_t e = sym ? launch_lw_sym(dim, v.pd, d, W, st, cg, *sym, qpart, pqrec, v.n_pad, s)
                     : launch_lw(dim, v, d, W, st, cg, qpart, pqrec, sp, s);
  if (e != hipSuccess) return e;
  if (dim == 2) {
    k_cg_update<2><<<nblk, 256, 0, s>>>(v, W, comp, n, qpart, slices, st, cg, part, nblk, pqrec, npq);
    k_cg_dir<2><<<nblk, 256, 0, s>>>(v, st, cg, part, nblk, tol * tol, max_steps);
  } else {
    k_cg_update<3><<<nblk, 256, 0, s>>>(v, W, comp, n, qpart, slices, st, cg, part, nblk, pqrec, npq);
    k_cg_dir<3><<<nblk, 256, 0, s>>>(v, st, cg, part, nblk, tol * tol, max_steps);
  }
  return hipGetLastError();
}

}  // namespace sl
