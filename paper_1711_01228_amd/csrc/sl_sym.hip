// Force pass over unordered pairs (Newton's third law), with the matrix cores
// doing the accumulation.
//
// F_i = sum_j c_ij (x_i - x_j), c_ij = (1/d)(1/r) - 1/d^2 = c_ji.  Written as
// F_i = (x_i - ref) S_i - sum_j c_ij (x_j - ref), S_i = sum_j c_ij, for a fixed
// reference point ref (vertex 0), the sums over j are matrix products C [X-ref, 1]
// with C generated on the fly.  Each unordered pair's c is computed once on the
// vector units and used by two MFMA products:
//   rows    D_i  += sum_j c_ij [x_j - ref, 1]      (v_mfma_f32_4x4x1_16b)
//   columns D'_j += sum_i c_ij [x_i - ref, 1]      (v_mfma_f32_16x16x4)
// A 64 x 64 block of pairs (row strip I, column strip J > I) is 16 sub-blocks of
// 16 x 16; a sub-block is 4 registers of c per lane.  In the rows' layout lane l,
// register s holds c(i = 4s + l%4, j = l/4), the A operand of the 16-block
// 4x4x1 product (rows stay in 64 FP32 accumulators, reduced over the 16 blocks
// and folded into FP64 every 16 column strips).  The columns use the same 4x4x1
// product on the same register with each 16-lane row transposed as a 4 x 4
// (bpermute): there lane l holds c(i = 4s + (l/4)%4, j = 4(l/16) + l%4), so a
// block's 4 lanes share i and the product accumulates over i into 4 columns per
// block; the 4 blocks of a row of lanes (one per i%4) are added with two
// rotations at the end of each 16-column sub-block.
// Diagonal blocks (J = I, 1/nb of the pairs) are left to k_sym_reduce, which
// evaluates each vertex's 63 pairs within its own strip directly.
//
// Work: a workgroup of 8 waves owns a panel of 8 row strips and a run of column
// strips J; each wave takes one strip, and loads the next strip's positions and
// distances while it computes the current one.  Rows accumulate in registers
// (FP32 per 16 column strips, then folded into FP64); every 4 strips the 8
// waves' column sums are added in wave order in LDS and written once per
// (panel, column) as FP32.
// k_sym_reduce adds, for each vertex, its row partials (in item order) and its
// column partials (in panel order) in FP64 and forms F.  All orders are fixed:
// results are bitwise repeatable.
//
// Distances are read from a copy of the upper triangle (I <= J) in the order the
// lanes consume them: per (I, J) 4 KiB, per column sub-block b 1 KiB, lane l's 16
// bytes hold d(i = 16a + 4s + l%4, j = 16b + l/4) at byte 4a + s.
#include "sl_device.h"

#include <algorithm>

namespace sl {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kPanel = 8;  // row strips (waves) per workgroup

__device__ __forceinline__ size_t tri_block(int I, int J, int nb) {
  return (size_t)I * nb - (size_t)I * (I - 1) / 2 + (size_t)(J - I);
}

// Component n of (p - ref) as an MFMA B operand: coordinates, then 1 (the row
// sum S), then 0.  All candidates are formed and one is selected (no branch, so
// the position is loaded whole).
template <int DIM>
__device__ __forceinline__ float b_operand(const typename VecT<DIM>::T& p, const typename VecT<DIM>::T& ref, int n) {
  const float c0 = p.x - ref.x, c1 = p.y - ref.y;
  float c2 = 1.f, c3 = 0.f;
  if constexpr (DIM == 3) {
    c2 = p.z - ref.z;
    c3 = 1.f;
  }
  const float lo = (n & 1) ? c1 : c0, hi = (n & 1) ? c3 : c2;
  return (n & 2) ? hi : lo;
}

// Reduce-scatter of 16 v4f registers over lane bits 5..2: afterwards lane l holds
// in R[0] the totals of register r = l >> 2 (summed over the 16 lanes that share
// l & 3).  Register index bits 3..0 follow lane bits 5..2.
__device__ __forceinline__ void reduce_scatter16(v4f (&R)[16], int lane) {
#pragma unroll
  for (int step = 0; step < 4; ++step) {
    const int bit = 5 - step;         // lane bit paired in this step
    const int half = 8 >> step;       // register pairs (r, r + half)
    const bool up = (lane >> bit) & 1;
#pragma unroll
    for (int r = 0; r < half; ++r) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float send = up ? R[r][v] : R[r + half][v];
        const float keep = up ? R[r + half][v] : R[r][v];
        R[r][v] = keep + __shfl_xor(send, 1 << bit, 64);
      }
    }
  }
}

// x from lane (l + R) mod 16 of the same row of 16 lanes (DPP row rotation).
template <int R>
__device__ __forceinline__ float rot16(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x120 + (16 - R), 0xf, 0xf, false));
}

template <int DIM>
__global__ __launch_bounds__(512) void k_force_sym(const uint8_t* __restrict__ dsym, const float* __restrict__ Xb,
                                                   size_t stride, const DevState* __restrict__ st,
                                                   const int4* __restrict__ items, double* __restrict__ Pi,
                                                   float* __restrict__ Pj, int nb, int n_pad) {
  using V = typename VecT<DIM>::T;
  constexpr int kGroup = 4;   // column strips between workgroup reductions of the column sums
  constexpr int kFold = 16;   // column strips between FP64 folds of the row sums
  __shared__ float2 lut[256];
  __shared__ float red[kGroup][kPanel][64][4];
  if (st->done) return;
  if (threadIdx.x < 256) {
    const float fb = (float)threadIdx.x;
    lut[threadIdx.x] = threadIdx.x ? make_float2(1.0f / fb, 1.0f / (fb * fb)) : make_float2(0.f, 0.f);
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
  const int4 it = items[blockIdx.x];
  const int panel = it.x, J0 = it.y, J1 = it.z, item = it.w;
  const int I = panel * kPanel + wave;
  const bool strip = I < nb;
  const V* __restrict__ X = reinterpret_cast<const V*>(Xb + (size_t)st->cur * stride);
  const V ref = X[0];
  // rows of strip I in the rows' layout (lane l: i = 16a + 4s + l%4), and the
  // columns' B operand (lane l holds component l%4 of row 16a + 4s + (l/4)%4)
  V xi[4][4];
  float Bi[4][4];
  // (a wave with no strip reads strip 0 and never uses it: every load is issued
  // on every lane, so none sits behind a branch)
  const size_t base = strip ? (size_t)I * 64 : 0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      xi[a][s] = X[base + 16 * a + 4 * s + (l & 3)];
      Bi[a][s] = b_operand<DIM>(X[base + 16 * a + 4 * s + ((l >> 2) & 3)], ref, l & 3);
    }
  }
  // lane that holds c(i = 4s + (l/4)%4, j = 4(l/16) + l%4) in the rows' layout
  // (lane 4 j + i%4): the 4 x 4 transpose of each row of 16 lanes
  const int col_src = 4 * ((l & 0x30) + 4 * (l & 3) + ((l >> 2) & 3));
  v4f D1[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) D1[r] = v4f{0.f, 0.f, 0.f, 0.f};
  double acc1[4] = {0.0, 0.0, 0.0, 0.0};
  // operands of the next column strip, loaded one strip ahead.  The loads are
  // issued on every path (a wave with no next block reads block (0, 0) and
  // strip J0, both in bounds), so the count of loads in flight is the same on
  // every path and the wait for the current strip leaves the next one in flight.
  V xn[4];
  uint4 qn[4];
#define SL_SYM_FETCH(JJ)                                                            \
  do {                                                                              \
    const int Jf = (JJ);                                                            \
    const bool use = strip && Jf > I && Jf < J1;                                    \
    const int Jl = use ? Jf : J0;                                                   \
    const uint8_t* blk = dsym + (use ? tri_block(I, Jf, nb) * 4096 : 0);            \
    _Pragma("unroll") for (int b = 0; b < 4; ++b) {                                  \
      xn[b] = X[(size_t)Jl * 64 + 16 * b + (l >> 2)];                               \
      qn[b] = reinterpret_cast<const uint4*>(blk + b * 1024)[l];                    \
    }                                                                               \
  } while (0)
  SL_SYM_FETCH(J0);
  __syncthreads();  // the weight table
  for (int J = J0; J < J1; ++J) {
    const bool active = strip && J > I;  // the diagonal block is k_sym_reduce's
    const int g = (J - J0) % kGroup;
    V xj[4];
    uint4 q[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      xj[b] = xn[b];
      q[b] = qn[b];
    }
    SL_SYM_FETCH(J + 1);
    if (active) {
      float Bj[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) Bj[b] = b_operand<DIM>(xj[b], ref, l & 3);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        // four independent column accumulators (one per s), added at the end
        v4f E[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) E[s] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int h = 0; h < 2; ++h) {  // rows 32h .. 32h + 31 of the strip: 8 pairs per lane
          float2 wt[8];
          float rinv[8], c[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int a = 2 * h + k / 4, s = k % 4;
            wt[k] = lut[byte_of(chunk_word(q[b], 4 * a), s)];
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int a = 2 * h + k / 4, s = k % 4;
            const float dx = xi[a][s].x - xj[b].x, dy = xi[a][s].y - xj[b].y;
            float r2 = fmaf(dx, dx, kTiny);
            r2 = fmaf(dy, dy, r2);
            if constexpr (DIM == 3) {
              const float dz = xi[a][s].z - xj[b].z;
              r2 = fmaf(dz, dz, r2);
            }
            rinv[k] = __builtin_amdgcn_rsqf(r2);
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) c[k] = fmaf(wt[k].x, rinv[k], -wt[k].y);
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int a = 2 * h + k / 4, s = k % 4;
            D1[4 * a + s] = __builtin_amdgcn_mfma_f32_4x4x1f32(c[k], Bj[b], D1[4 * a + s], 0, 0, 0);
          }
          // columns: block (i%4, j/4) accumulates c(i, j) (x_i - ref)[n] over its rows i
          int u[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) u[k] = __builtin_amdgcn_ds_bpermute(col_src, __float_as_int(c[k]));
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int a = 2 * h + k / 4, s = k % 4;
            E[s] = __builtin_amdgcn_mfma_f32_4x4x1f32(__int_as_float(u[k]), Bi[a][s], E[s], 0, 0, 0);
          }
        }
        v4f D2 = (E[0] + E[1]) + (E[2] + E[3]);
        // add the 4 blocks of each row of 16 lanes (lane bits 3..2 = i%4): rotate
        // by 8, then by 4, within the row; lanes l%16 < 4 end with the totals
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          D2[v] += rot16<8>(D2[v]);
          D2[v] += rot16<4>(D2[v]);
        }
        // lane l (l%16 < 4), register v: column 16 b + 4 (l / 16) + v, component l % 4
        if ((l & 15) < 4) {
#pragma unroll
          for (int v = 0; v < 4; ++v) red[g][wave][16 * b + 4 * (l >> 4) + v][l & 15] = D2[v];
        }
      }
    } else if ((l & 15) < 4) {
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[g][wave][16 * b + 4 * (l >> 4) + v][l & 15] = 0.f;
    }
    if (g == kGroup - 1 || J + 1 == J1) {
      // the 8 waves' column sums of the last g + 1 strips, in wave order
      __syncthreads();
      const int Jb = J - g;
      for (int e = threadIdx.x; e < (g + 1) * 256; e += 512) {
        const int gg = e >> 8, j = (e >> 2) & 63, n = e & 3;
        float t = 0.f;
#pragma unroll
        for (int w = 0; w < kPanel; ++w) t += red[gg][w][j][n];
        Pj[((size_t)panel * n_pad + (size_t)(Jb + gg) * 64 + j) * 4 + n] = t;
      }
      __syncthreads();
    }
    if (((J - J0) % kFold) == kFold - 1 || J + 1 == J1) {
      // fold the rows' FP32 sums into FP64
      if (strip) {
        reduce_scatter16(D1, l);
#pragma unroll
        for (int v = 0; v < 4; ++v) acc1[v] += (double)D1[0][v];
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) D1[r] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  }
  if (strip) {
    // lane l: rows 4 (l >> 2) + v of strip I, component l & 3
    double* out = Pi + ((size_t)item * kPanel * 64 + (size_t)wave * 64) * 4;
#pragma unroll
    for (int v = 0; v < 4; ++v) out[(4 * (l >> 2) + v) * 4 + (l & 3)] = acc1[v];
  }
#undef SL_SYM_FETCH
}

// F_i = (x_i - ref) S_i - D_i from the row partials of the items of i's panel
// (in item order), the column partials of the panels at or above i's strip (in
// panel order) and the pairs of i's own strip (the diagonal block, evaluated
// here in order of j), into force slice 0.
template <int DIM>
__global__ __launch_bounds__(256) void k_sym_reduce(const double* __restrict__ Pi, const float* __restrict__ Pj,
                                                    const int32_t* __restrict__ panel_items,
                                                    const uint8_t* __restrict__ dsym, const float* __restrict__ Xb,
                                                    size_t stride, const DevState* __restrict__ st,
                                                    double* __restrict__ fpart, int nb, int n_pad) {
  using V = typename VecT<DIM>::T;
  if (st->done) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n_pad) return;
  const int strip = i / 64, panel = strip / kPanel, row = i % (kPanel * 64);
  const V* __restrict__ X = reinterpret_cast<const V*>(Xb + (size_t)st->cur * stride);
  const V x = X[i], ref = X[0];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  {
    // diagonal block: d(i, j) sits at byte (j/16) 1024 + (4 (j%16) + i%4) 16 + 4 ((i%64)/16) + (i/4)%4
    const uint8_t* blk = dsym + tri_block(strip, strip, nb) * 4096;
    const int ia = (i & 63) >> 4, is = (i >> 2) & 3, i4 = i & 3;
    for (int jj = 0; jj < 64; ++jj) {
      const int dv = blk[(jj >> 4) * 1024 + (4 * (jj & 15) + i4) * 16 + 4 * ia + is];
      if (dv == 0) continue;  // i itself and padding
      const V xj = X[strip * 64 + jj];
      const float fd = (float)dv, inv = 1.0f / fd, w = 1.0f / (fd * fd);
      const float dx = x.x - xj.x, dy = x.y - xj.y;
      float r2 = fmaf(dx, dx, kTiny);
      r2 = fmaf(dy, dy, r2);
      if constexpr (DIM == 3) {
        const float dz = x.z - xj.z;
        r2 = fmaf(dz, dz, r2);
      }
      const double c = (double)fmaf(inv, __builtin_amdgcn_rsqf(r2), -w);
      acc[0] += c * ((double)xj.x - (double)ref.x);
      acc[1] += c * ((double)xj.y - (double)ref.y);
      if constexpr (DIM == 3) acc[2] += c * ((double)xj.z - (double)ref.z);
      acc[DIM] += c;
    }
  }
  for (int q = panel_items[panel]; q < panel_items[panel + 1]; ++q) {
    const double* p = Pi + ((size_t)q * kPanel * 64 + row) * 4;
#pragma unroll
    for (int n = 0; n <= DIM; ++n) acc[n] += p[n];
  }
  for (int p = 0; p <= panel; ++p) {
    const float* c = Pj + ((size_t)p * n_pad + i) * 4;
#pragma unroll
    for (int n = 0; n <= DIM; ++n) acc[n] += (double)c[n];
  }
  const double S = acc[DIM];
  fpart[i] = ((double)x.x - (double)ref.x) * S - acc[0];
  fpart[(size_t)n_pad + i] = ((double)x.y - (double)ref.y) * S - acc[1];
  if constexpr (DIM == 3) fpart[2 * (size_t)n_pad + i] = ((double)x.z - (double)ref.z) * S - acc[2];
}

// The upper triangle of d in the symmetric pass's order (see above), one
// (I, J) block per workgroup.
__global__ __launch_bounds__(256) void k_build_sym(const uint8_t* __restrict__ d, uint8_t* __restrict__ dsym, int nb,
                                                   int ng) {
  const int J = blockIdx.x, I = blockIdx.y;
  if (J < I || J >= nb) return;
  uint8_t* out = dsym + tri_block(I, J, nb) * 4096;
  for (int e = threadIdx.x; e < 4096; e += 256) {
    const int b = e / 1024, l = (e / 16) % 64, a = (e % 16) / 4, s = e % 4;
    const int i = I * 64 + 16 * a + 4 * s + (l & 3), j = J * 64 + 16 * b + (l >> 2);
    out[e] = d[tile_offset(i, j, ng)];
  }
}

}  // namespace

SymSplit make_sym_split(int n_pad, int chunk) {
  SymSplit sp;
  sp.nb = n_pad / 64;
  sp.npanels = (sp.nb + kPanel - 1) / kPanel;
  sp.panel_items.assign(sp.npanels + 1, 0);
  for (int p = 0; p < sp.npanels; ++p) {
    for (int J0 = p * kPanel; J0 < sp.nb; J0 += chunk) {
      const int J1 = std::min(J0 + chunk, sp.nb);
      sp.items.push_back(make_int4(p, J0, J1, (int)sp.items.size()));
    }
    sp.panel_items[p + 1] = (int)sp.items.size();
  }
  return sp;
}

size_t sym_bytes(int n_pad) {
  const size_t nb = n_pad / 64;
  return nb * (nb + 1) / 2 * 4096;
}

hipError_t launch_build_sym(const uint8_t* d, uint8_t* dsym, int n_pad, int ng, hipStream_t s) {
  const int nb = n_pad / 64;
  k_build_sym<<<dim3(nb, nb), 256, 0, s>>>(d, dsym, nb, ng);
  return hipGetLastError();
}

hipError_t launch_force_sym(int dim, const uint8_t* dsym, const float* Xb, size_t stride, const DevState* st,
                            const int4* items, int nitems, const int32_t* panel_items, double* Pi, float* Pj,
                            double* fpart, int n_pad, hipStream_t s) {
  const int nb = n_pad / 64;
  if (dim == 2) {
    k_force_sym<2><<<nitems, 512, 0, s>>>(dsym, Xb, stride, st, items, Pi, Pj, nb, n_pad);
    k_sym_reduce<2><<<(n_pad + 255) / 256, 256, 0, s>>>(Pi, Pj, panel_items, dsym, Xb, stride, st, fpart, nb, n_pad);
  } else {
    k_force_sym<3><<<nitems, 512, 0, s>>>(dsym, Xb, stride, st, items, Pi, Pj, nb, n_pad);
    k_sym_reduce<3><<<(n_pad + 255) / 256, 256, 0, s>>>(Pi, Pj, panel_items, dsym, Xb, stride, st, fpart, nb, n_pad);
  }
  return hipGetLastError();
}

}  // namespace sl
