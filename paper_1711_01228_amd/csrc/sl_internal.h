// Internal declarations shared by the kernels (sl_kernels.hip) and the host
// runtime (sl_api.hip) of libsorlayout.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <vector>

namespace sl {

// ---------------------------------------------------------------------------
// Device data layout
//
//   n_pad  = n rounded up to 64; rows and columns past n are padding.
//   d      one byte per ordered pair (i, j): the hop distance d_ij, 0 for i = j
//          or no path.  Tile-major: a tile is 64 rows x 16 columns stored as
//          64 lane-chunks of 16 bytes, so a wave whose lane l owns row
//          64*rb + l reads one tile as one contiguous 1 KiB load:
//            offset(i, j) = ((i/64) * NG + j/16) * 1024 + (i%64) * 16 + j%16,
//          NG = n_pad / 16 column groups per row block.
//   X      iterates as float2 (dim 2) or float4 with w = 0 (dim 3), n_pad
//          entries each, padding at the origin.  Three buffers rotate: the
//          current iterate, X^H and X~; DevState::cur names the current one.
//   E      the extrapolation step e_i = x~_i - x^H_i as stored (same format),
//          read by the safeguard pass.
// ---------------------------------------------------------------------------
constexpr int kWeightedMaxN = 16384;  // weighted graphs: one source's distance row fits in LDS
constexpr int kRowBlock = 64;   // rows per wave (one per lane)
constexpr int kColGroup = 16;   // columns per 16-byte lane chunk
constexpr int kTileBytes = kRowBlock * kColGroup;

__host__ __device__ inline size_t tile_offset(int64_t i, int64_t j, int64_t ng) {
  return (size_t)(((i / kRowBlock) * ng + j / kColGroup) * kTileBytes + (i % kRowBlock) * kColGroup + j % kColGroup);
}

// Iteration state kept in device memory so that a captured graph of several
// iterations can be replayed: every kernel reads `done` and returns at once
// when it is set, and reads `cur` to find the current iterate.
struct DevState {
  int32_t cur;        // buffer index of X^k (0..2)
  int32_t iter;       // iterations completed
  int32_t done;       // 1: converged, max_iter reached or numeric failure
  int32_t converged;
  int32_t rejected;
  int32_t status;     // 0 or SL_ENUMERIC
  int32_t max_iter;
  int32_t prev;       // buffer index of the iterate the last completed iteration started from
  double residual;
  double last_df;
  double stress;      // f of the last evaluated placement (stress passes)
  double omega_used;  // paper's factor of the last iteration
  double enum_c;      // enumerating: factor picked by the last select
  int32_t enum_pending;  // enumerating: X~ = X^H + enum_c * step is still to be formed
  int32_t need_force;    // fused safeguard: X~ was rejected, the force at X^H is still to come
  int32_t need_exact;    // bounded safeguard: the bounds left the sign of f(X~) - f(X^H) open,
                         // the exact pass and the second select are still to come
  int32_t exact_next;    // bounded safeguard: the next extrapolating iteration sums the exact
                         // difference in its fused pass (the bounds left the last one open)
  double bound_u, bound_l;  // bounded safeguard: U >= f(X~) - f(X^H) >= L of this iteration
};

// Columns of a trace row (SL_TRACE_COLS of sorlayout.h).
constexpr int kTraceCols = 7;

constexpr int kEnumCandidates = 18;  // paper's factors 0.5, 1.0, ..., 9.0 (0 = keep X^H)

// Scalars every kernel of the loop needs, passed by value.
struct LoopParams {
  int32_t n, n_pad, ng, nrb, slices, groups_per_slice;
  double omega_p;     // paper's relaxation factor = omega - 1
  double tol;
  int32_t safeguard;  // evaluate f(X~) - f(X^H) and select
  int32_t stress;     // accumulate f(X^k) in the force pass
  int32_t enumerate;  // SL_OMEGA_ENUM
  int32_t pad;
  const double* omega_sched;  // device, paper's factors per iteration, or nullptr
  const float* omega_vertex;  // device, classical factors per vertex, or nullptr
  // exact step: X^H = Y, the conjugate-gradient solution (double, column c at
  // c * n_pad); nullptr for the Jacobi step
  const double* exact_y;
  int32_t sym;   // the force pass runs over unordered pairs (F in slice 0; slices = 1)
  int32_t fuse;  // the safeguard rides on the next iteration's force pass (at X~)
  // the fused pass forms bounds U >= f(X~) - f(X^H) >= L instead of the
  // difference itself; the exact pass runs only when they leave its sign open
  int32_t bounds;
  int32_t pad2;
};

// ---------------------------------------------------------------------------
// Exact step H (eq. 5 solved by preconditioned conjugate gradients)
// ---------------------------------------------------------------------------
struct CgVectors {
  int32_t n_pad, pad;
  double *y, *r, *z;  // dim x n_pad each (column c at c * n_pad)
  double* pd;         // search direction as double2 (dim 2) / double4 (dim 3), n_pad entries
};

// Step counters: `ja` is read by the update and direction kernels and copied
// from `jb` by the matvec; `jb` is written by the direction kernel.  No kernel
// reads a field it writes, so blocks of one launch never race on them.
struct CgState {
  int32_t ja, jb;
  int32_t done;   // 1: converged or step limit; the remaining kernels return
  int32_t iters;  // steps taken for the current H
  double rel;     // ||r|| / ||r_0|| when the solve stopped
};

inline int cg_blocks(int n_pad) { return (n_pad + 255) / 256; }
// Partial-sum records (8 doubles per block): two rotating slots of
// [r.z, ||r||^2] per column, the initial slot, then one p.q record per matvec block.
constexpr int kCgInitial = 2;
constexpr int kCgSlots = 3;

hipError_t launch_components(const uint8_t* d, int32_t* comp, int n, int n_pad, int ng, hipStream_t s);
hipError_t launch_cg_init(int dim, const CgVectors& v, const double* fpart, int slices, const double* W,
                          const int32_t* comp, int n, const float* Xb, size_t stride, const DevState* st, CgState* cg,
                          double* part, hipStream_t s);


// Work split of the all-pairs passes for a graph of n_pad vertices.
struct Split {
  int nrb;              // row blocks (waves per column slice)
  int ng;               // column groups
  int slices;           // column slices S
  int groups_per_slice; // column groups per slice
  int blocks_x;         // workgroups along rows (4 waves each)
};
Split make_split(int n_pad);
struct LwSym;
// One step: matvec (with the stop test), p/q update, Y/r/z update; the matvec
// over unordered pairs when `sym` is given.
hipError_t launch_cg_step(int dim, const CgVectors& v, const uint8_t* d, const double* W, const int32_t* comp, int n,
                          const DevState* st, CgState* cg, double* part, double* qpart, const Split& sp, double tol,
                          int max_steps, const LwSym* sym, hipStream_t s);
// Force pass over unordered pairs (sl_sym.hip): work items (panel of 8 row
// strips, first and end column strip, item index), the items of each panel
// contiguous.
struct SymSplit {
  int nb = 0, npanels = 0;
  std::vector<int4> items;
  std::vector<int32_t> panel_items;  // npanels + 1 offsets into items
};
SymSplit make_sym_split(int n_pad);
int sym_rows_per_item();  // rows of one work item (its panel of row strips)
// Writes F into force slice 0 of fpart (Pi: items x sym_rows_per_item() x dim floats, Pj:
// panels x n_pad x dim floats of partial sums); cond: only when the state asks
// for the force again (after a rejection).
hipError_t launch_force_sym(int dim, int cond, const uint8_t* d, const float* df, const float* Xb, size_t stride,
                            const DevState* st, const int4* items, int nitems, const int32_t* panel_items, float* Pi,
                            float* Pj, double* fpart, int n_pad, hipStream_t s);
// The same pass at X~ with the bounds of the safeguard summed in: B and C of
// each item into sgpart[2 item], sgpart[2 item + 1], and sum e_i . F_i of each
// reduction workgroup into edot (sym_reduce_blocks(n_pad) doubles).  With
// `exact` the difference f(X~) - f(X^H) itself too, into sgpart[2 nitems + item].
// With `gated` the launch does work only in the iterations the state gives to
// it (DevState::exact_next: the exact variant, else the bounds alone).  The
// reduction into fpart and edot follows the pass (kSymReducePass), is left
// out (kSymReduceNone), or runs in every iteration that is not done
// (kSymReduceAny: after the second of the two gated variants, one of which
// runs in each iteration).
constexpr int kSymReducePass = 0, kSymReduceNone = 1, kSymReduceAny = 2;
hipError_t launch_force_sym_sg(int dim, const LoopParams& lp, int exact, int gated, int reduce, const uint8_t* d,
                               const float* df,
                               const float* Xb, size_t stride, const float* Eb, const DevState* st, const int4* items,
                               int nitems, const int32_t* panel_items, float* Pi, float* Pj, double* sgpart,
                               double* fpart, double* edot, int n_pad, hipStream_t s);
unsigned sym_reduce_blocks(int n_pad);
// One application of L^W to p (also used by the profiler).
hipError_t launch_lw(int dim, const CgVectors& v, const uint8_t* d, const double* W, const DevState* st, CgState* cg,
                     double* qpart, double* pqrec, const Split& sp, hipStream_t s);
// The same over unordered pairs (sl_sym.hip): the force pass's work items, FP64
// row partials Pi (items x sym_rows_per_item() x dim) and column partials Pj
// (panels x n_pad x dim); q into slice 0 of qpart and lw_sym_reduce_blocks(n_pad)
// p.q records into pqrec.
struct LwSym {
  const int4* items = nullptr;
  int nitems = 0;
  const int32_t* panel_items = nullptr;
  double* Pi = nullptr;
  double* Pj = nullptr;
};
unsigned lw_sym_reduce_blocks(int n_pad);
hipError_t launch_lw_sym(int dim, const double* pd, const uint8_t* d, const double* W, const DevState* st, CgState* cg,
                         const LwSym& ls, double* qpart, double* pqrec, int n_pad, hipStream_t s);

// ---- launchers (sl_kernels.hip); all enqueue on `s` and return the launch status
hipError_t launch_fill_u8(uint8_t* p, size_t bytes, hipStream_t s);
// ---- distances and weights (sl_apsp.hip)
int bfs_sources_per_sweep();  // sources searched together (bits per vertex)
int bfs_words();              // 64-bit words per vertex in the BFS buffers
int bfs_slots();              // level bitmaps kept (levels per batch)
// slots: bfs_slots() buffers of n * bfs_words() words; slot l % bfs_slots()
// holds the sources that first reach each vertex at level l >= 1 (the sources
// themselves, level 0, are formed where needed).  masks: bfs_slots() buffers
// of n words; bit c of mask l % bfs_slots() of v is set iff 16-byte chunk c
// of v's level-l row is not zero, and only those chunks are written: a chunk
// whose bit is clear holds stale bytes and is read as zero.  Level l writes
// every vertex's mask; neither buffer needs clearing.
// Runs of the gather: int4 (first CSR entry, count, row of that entry, 0),
// count 1 .. bfs_run_entries(): whole rows of at most that many entries packed
// together (a run never splits one).  Every other row is listed in longrows as
// int4 (vertex, first CSR entry, degree, 0): first the nbig rows of degree above
// bfs_mid_max_degree() (a workgroup each), then the nmid others (degree up to
// that, or 0: a wave each).
int bfs_run_entries();
int bfs_mid_max_degree();
// pairs (nruns * bfs_run_entries() int2): the runs' entries as (neighbour, row),
// (-1, -1) past a run's count; row_ptr and col_idx on the device.
hipError_t launch_bfs_pairs(const int4* runs, int nruns, const int64_t* row_ptr, const int32_t* col_idx, int2* pairs,
                            hipStream_t s);
// One BFS level (1 .. 256) of the sweep from sources base ...  flags[0 .. 256]:
// flags[l] != 0 iff level l found a new vertex (flags[0]: the sources); a level
// after an empty one does nothing.
hipError_t launch_bfs_level(const int2* pairs, int nruns, const int4* longrows, int nbig, int nmid,
                            const int32_t* col_idx, const uint64_t* slots, uint64_t* masks, int n, int base,
                            int level, int32_t* flags, hipStream_t s);
// `sweeps` flag rows of `stride` ints: [s][0] = 1, the rest 0.
hipError_t launch_bfs_flags(int32_t* flags, int sweeps, int stride, hipStream_t s);
// Weight partials of the stores: bfs_weight_partials() x n_pad doubles, zero
// before the first sweep; W_v = their sum in order (0 past n).
int bfs_weight_partials();
hipError_t launch_weights_from_partials(const double* wq, double* W, int n, int n_pad, hipStream_t s);
// Levels l0 .. l1 (l1 - l0 < bfs_slots(), l1 <= 255) of the sweep from sources
// base .. base + bfs_sources_per_sweep() - 1 into d; the batch starting at
// level 1 writes every byte of the sweep's columns (below n_pad) in all rows.
// The weights d^-2 of the pairs found at levels >= count_from are added into
// the partials wq.
hipError_t launch_bfs_store(const uint64_t* slots, const uint64_t* masks, const int32_t* flags, uint8_t* d,
                            double* wq, int n, int n_pad, int base, int l0, int l1, int count_from, hipStream_t s);
// W from d (or df); wpart: scratch of sp.slices * n_pad doubles.
hipError_t launch_weights(const uint8_t* d, const float* df, double* W, double* wpart, const Split& sp, int n,
                          hipStream_t s);
// Weighted graphs: FP32 shortest-path distances (tile-major, 0 = no path) and
// trees (pred[s][v], row-major int32), then the lower triangle := the upper.
// erow: the row of every CSR entry.
hipError_t launch_wsssp(const int32_t* erow, const int32_t* col_idx, const float* len, int64_t nnz, int n, int ng,
                        float* df, int32_t* pred, hipStream_t s);
hipError_t launch_wsym(float* df, int n_pad, int ng, hipStream_t s);
// Reverse mode (sl_diff.hip).
hipError_t launch_grad_in(const float* G, double* gb, int n, int n_pad, int dim, hipStream_t s);
hipError_t launch_grad_out(const double* gb, float* G, int n, int n_pad, int dim, hipStream_t s);
hipError_t launch_stress_grad_out(const double* fpart, int slices, int n, int n_pad, int dim, float* G,
                                  hipStream_t s);
hipError_t launch_save(const float* Xb, size_t stride, const DevState* st, float* dst, hipStream_t s);
// One backward iteration at X^k (Xk, iterate layout) given the force sums at X^k
// in fpart: gb += Xbar; with Dbar, dL/dd of every row added into it.  The
// adjoint pass reuses apart (may be fpart).
hipError_t launch_adjoint_step(int dim, const uint8_t* d, const float* df, const float* Xk, const double* fpart,
                               int fslices, const double* W, double a, double* gb, float* gvec, float* wbar,
                               double* apart, const struct Split& sp, int n_pad, hipStream_t s);
// dL/dd of a segment of nk iterations into Dbar, from the iterates (segX) and
// the adjoint vectors (gseg: nk x stride floats, wseg: nk x n_pad) of each.
hipError_t launch_dbar_segment(int dim, const uint8_t* d, const float* df, const float* segX, size_t stride,
                               const float* gseg, const float* wseg, int nk, float* Dbar, const struct Split& sp,
                               int n_pad, hipStream_t s);
// dL/dlen per CSR entry from Dbar through the shortest-path trees (S: n x n
// floats of scratch, G: nnz doubles of scratch, erow: source row of each entry).
hipError_t launch_edge_grad(const float* Dbar, float* S, const int64_t* row_ptr, const int32_t* col_idx,
                            const int32_t* erow, const int32_t* pred, double* G, float* glen, int n, int64_t nnz,
                            int n_pad, int ng, hipStream_t s);
hipError_t launch_pack_in(const float* X, float* Xb, int n, int n_pad, int dim, hipStream_t s);
hipError_t launch_pack_out(const float* Xb, const DevState* st, size_t stride, float* X, int n, int dim,
                           hipStream_t s);
// Distances are bytes (d) or, for weighted graphs, floats (df); the other pointer is null.
hipError_t launch_force(int dim, bool stress, const uint8_t* d, const float* df, const float* Xb, size_t stride,
                        const DevState* st, double* fpart, double* spart, const Split& sp, int n_pad,
                        hipStream_t s);
// The force pass at X~ with the safeguard sums of the same iteration (one
// double per workgroup into sgpart: slices * blocks_x of them).
hipError_t launch_force_sg(int dim, const LoopParams& lp, const uint8_t* d, const float* df, const float* Xb,
                           size_t stride, const float* Eb, const DevState* st, double* fpart, double* sgpart,
                           const Split& sp, hipStream_t s);
// The force pass at X^k if the last select rejected X~ in a fused iteration.
hipError_t launch_force_cond(int dim, const uint8_t* d, const float* df, const float* Xb, size_t stride,
                             const DevState* st, double* fpart, const Split& sp, int n_pad, hipStream_t s);
hipError_t launch_update(int dim, const LoopParams& p, const double* fpart, const double* spart,
                         const double* W, float* Xb, size_t stride, float* Eb, const DevState* st, double* red,
                         hipStream_t s);
// Work items (row block, first column group, end group, 0) of the safeguard
// pass: the upper triangle in equal runs of column groups.
std::vector<int4> triangle_items(const Split& sp);
// gate: run only when the state asks for the exact difference (need_exact).
hipError_t launch_sgdelta(int dim, const uint8_t* d, const float* df, const float* Xb, size_t stride,
                          const float* Eb, const int4* items, int nitems, const DevState* st, double* sgpart,
                          const Split& sp, hipStream_t s, int gate = 0);
// Modes of the select kernel.
constexpr int kSelectPlain = 0;   // sgpart: nsg partial sums of f(X~) - f(X^H)
constexpr int kSelectBounds = 1;  // sgpart: (B, C) of nsg items, edot: nedot partial sums of e . F, and
                                  // after the exact variant (exact_next) the nsg differences from
                                  // sgpart + 2 nsg; decides from those, from U and L, or leaves the
                                  // iteration to kSelectExact (need_exact)
constexpr int kSelectExact = 2;   // only after kSelectBounds left the sign open: sgpart as kSelectPlain
hipError_t launch_select(int dim, const LoopParams& p, const double* red, int nred, const double* sgpart,
                         int nsg, DevState* st, double* trace, hipStream_t s, int mode = kSelectPlain,
                         const double* edot = nullptr, int nedot = 0);
hipError_t launch_sgdelta_enum(int dim, const uint8_t* d, const float* Xb, size_t stride, const float* Eb,
                               const int4* items, int nitems, const DevState* st, double* sgpart, const Split& sp,
                               hipStream_t s);
hipError_t launch_apply_enum(const float* Eb, float* Xb, size_t stride, const DevState* st, int n, int dim,
                             hipStream_t s);
hipError_t launch_record(const float* Xb, size_t stride, const DevState* st, float* xtrace, int n, int dim,
                         hipStream_t s);
hipError_t launch_stress_sum(double* spart, int slices, int n_pad, DevState* st, hipStream_t s);
hipError_t launch_gather_rows(const uint8_t* d, const float* df, const int32_t* rows, int nrows, int n, int ng,
                              float* out, hipStream_t s);

// ---------------------------------------------------------------------------
// Batched layouts: many independent graphs of at most kBatchMaxN vertices.
// One persistent kernel: each workgroup takes the next graph from a queue
// (largest first) and runs its whole layout with the iterates in LDS.
// ---------------------------------------------------------------------------
constexpr int kBatchMaxN = 1024;
constexpr int kBatchMaxPartial = 2048;  // bound on slices * n_pad of one graph
constexpr int kBatchClasses = kBatchMaxN / kRowBlock;  // size classes n_pad = 64, 128, ..., 1024

struct BatchGraph {
  int32_t n, n_pad;
  int32_t slices;   // column slices of the all-pairs passes (tuned per size class)
  int32_t pad;
  int64_t d_off;    // byte offset of the graph's tile-major distance block
  int64_t v_off;    // first vertex of the graph in the concatenated arrays
  int64_t w_off;    // first entry of its n_pad weight sums
};

struct BatchResult {
  int32_t iterations, converged, rejected, status;
  double residual, stress;
};

struct BatchParams {
  double omega_p, tol;
  int32_t max_iter, safeguard;
};

// Column slices that give every wave of a `threads` workgroup a unit, within
// the LDS budget of the force partials (the default of a batch plan).
__host__ __device__ inline int batch_default_slices(int n_pad, int threads) {
  const int nrb = n_pad / kRowBlock, ng = n_pad / kColGroup, nw = threads / 64;
  int s = nw / nrb > 1 ? nw / nrb : 1;
  s = s < ng ? s : ng;
  s = s < kBatchMaxPartial / n_pad ? s : kBatchMaxPartial / n_pad;
  return s > 1 ? s : 1;
}

// Workgroups of a batched layout launch: the LDS of one graph (~78 KiB in 2-D,
// ~127 KiB in 3-D) allows two, or one, per CU.
inline int batch_layout_blocks(int dim, int cus, int count) {
  const int per_cu = dim == 2 ? 2 : 1;
  const int b = count < cus * per_cu ? count : cus * per_cu;
  return b > 1 ? b : 1;
}

hipError_t launch_batch_reset(int32_t* queue, hipStream_t s);
// Zero `bytes` bytes at p (16-byte aligned) with a kernel, not a memset node.
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_batch_distances(int threads, int blocks, const BatchGraph* graphs, const int32_t* order, int count,
                                  int32_t* queue, const int64_t* row_ptr, const int32_t* col_idx, uint8_t* d,
                                  double* W, int32_t* status, hipStream_t s);
hipError_t launch_batch_layout(int dim, int threads, int blocks, const BatchGraph* graphs, const int32_t* order,
                               int count, int32_t* queue, const uint8_t* d, const double* W, float* X,
                               BatchResult* res, const BatchParams& p, hipStream_t s);
bool batch_threads_supported(int threads);

}  // namespace sl
