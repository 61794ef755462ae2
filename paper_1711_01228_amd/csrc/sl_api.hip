// Host runtime of libsorlayout: argument validation, plan construction
// (distances and weights on the device), the iteration driver with
// device-side stopping and captured HIP graphs, and the C ABI of sorlayout.h.
#include "sorlayout.h"
#include "sl_internal.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <thread>
#include <vector>

using namespace sl;

static_assert(SL_TRACE_COLS == kTraceCols, "trace row layout");

namespace {

// The calling thread's last error message: a fixed buffer, so that reporting an
// error allocates nothing.
struct ErrorText {
  char text[512] = {0};
  void clear() { text[0] = 0; }
  const char* c_str() const { return text; }
};
thread_local ErrorText g_err;

sl_status fail(sl_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err.text, sizeof g_err.text, fmt, ap);
  va_end(ap);
  return st;
}

sl_status hip_fail(hipError_t e, const char* what) {
  const sl_status st = (e == hipErrorOutOfMemory) ? SL_ENOMEM : SL_EDEVICE;
  return fail(st, "%s: %s", what, hipGetErrorString(e));
}

// Every C entry point runs its body through this, so that no C++ exception
// (a host container that cannot grow, say) crosses the C ABI: it becomes a
// status and a message instead.
template <class F>
sl_status guarded(F&& body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return fail(SL_ENOMEM, "host allocation failed");
  } catch (const std::exception& x) {
    return fail(SL_EDEVICE, "host runtime error: %s", x.what());
  } catch (...) {
    return fail(SL_EDEVICE, "host runtime error");
  }
}

#define HIP_TRY(expr, what)                       \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// ---------------------------------------------------------------------------
// Host-side validation (no HIP calls)
// ---------------------------------------------------------------------------
// Edge lengths: positive, finite, the same on both entries of an edge.
sl_status check_lengths(const sl_graph* g, const float* len) {
  for (int64_t e = 0; e < g->nnz; ++e)
    if (!(std::isfinite(len[e]) && len[e] > 0.f))
      return fail(SL_EINVAL, "edge_len[%lld] is not a positive finite number", (long long)e);
  for (int64_t v = 0; v < g->n; ++v)
    for (int64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
      const int32_t u = g->col_idx[e];
      for (int64_t f = g->row_ptr[u]; f < g->row_ptr[u + 1]; ++f)
        if (g->col_idx[f] == v && len[f] != len[e])
          return fail(SL_EINVAL, "edge (%lld, %d) has two different lengths", (long long)v, u);
    }
  if (g->n > kWeightedMaxN)
    return fail(SL_ENOTSUP, "weighted graphs are limited to %d vertices (n = %d)", kWeightedMaxN, g->n);
  return SL_OK;
}

sl_status check_graph(const sl_graph* g) {
  if (!g) return fail(SL_EINVAL, "graph is NULL");
  if (g->n < 0) return fail(SL_EINVAL, "n = %d is negative", g->n);
  const int64_t n = g->n;
  if (n == 0) {
    if (g->nnz != 0) return fail(SL_EINVAL, "n = 0 but nnz = %lld", (long long)g->nnz);
    return SL_OK;
  }
  if (!g->row_ptr) return fail(SL_EINVAL, "row_ptr is NULL");
  if (g->nnz < 0) return fail(SL_EINVAL, "nnz is negative");
  if (g->nnz > 0 && !g->col_idx) return fail(SL_EINVAL, "col_idx is NULL");
  if (g->row_ptr[0] != 0) return fail(SL_EINVAL, "row_ptr[0] = %lld, expected 0", (long long)g->row_ptr[0]);
  for (int64_t v = 0; v < n; ++v)
    if (g->row_ptr[v + 1] < g->row_ptr[v])
      return fail(SL_EINVAL, "row_ptr decreases at row %lld", (long long)v);
  if (g->row_ptr[n] != g->nnz)
    return fail(SL_EINVAL, "row_ptr[n] = %lld differs from nnz = %lld", (long long)g->row_ptr[n], (long long)g->nnz);
  if (g->nnz > (int64_t)INT32_MAX * 2) return fail(SL_EINVAL, "nnz too large");
  // sorted copy of every row: range, self loops, duplicates, symmetry
  std::vector<int32_t> cols(g->col_idx, g->col_idx + g->nnz);
  for (int64_t v = 0; v < n; ++v) {
    const int64_t a = g->row_ptr[v], b = g->row_ptr[v + 1];
    for (int64_t e = a; e < b; ++e) {
      const int32_t u = cols[e];
      if (u < 0 || u >= n) return fail(SL_EINVAL, "row %lld has neighbour %d outside [0, n)", (long long)v, u);
      if (u == v) return fail(SL_EINVAL, "self loop at vertex %lld", (long long)v);
    }
    std::sort(cols.begin() + a, cols.begin() + b);
    for (int64_t e = a + 1; e < b; ++e)
      if (cols[e] == cols[e - 1])
        return fail(SL_EINVAL, "duplicate edge (%lld, %d)", (long long)v, cols[e]);
  }
  for (int64_t v = 0; v < n; ++v) {
    for (int64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
      const int32_t u = cols[e];
      if (!std::binary_search(cols.begin() + g->row_ptr[u], cols.begin() + g->row_ptr[u + 1], (int32_t)v))
        return fail(SL_EINVAL, "graph is not symmetric: (%lld, %d) has no reverse entry", (long long)v, u);
    }
  }
  if (g->edge_len) return check_lengths(g, g->edge_len);
  return SL_OK;
}

sl_status check_options(const sl_options* o) {
  if (!o) return fail(SL_EINVAL, "options are NULL");
  if (o->dim != 2 && o->dim != 3) return fail(SL_EINVAL, "dim = %d, expected 2 or 3", o->dim);
  if (!(std::isfinite(o->omega) && o->omega > 0.0 && o->omega <= 16.0))
    return fail(SL_EINVAL, "omega = %g outside (0, 16]", o->omega);
  if (!(o->tol >= 0.0)) return fail(SL_EINVAL, "tol = %g must be >= 0", o->tol);
  if (o->max_iter < 0) return fail(SL_EINVAL, "max_iter = %d is negative", o->max_iter);
  if (o->safeguard != 0 && o->safeguard != 1) return fail(SL_EINVAL, "safeguard must be 0 or 1");
  if (o->flags & ~(SL_FLAG_TRACE_STRESS | SL_FLAG_NO_GRAPH | SL_FLAG_SYM_FORCE | SL_FLAG_SEPARATE_SAFEGUARD |
                   SL_FLAG_ORDERED_FORCE | SL_FLAG_NO_FINAL_STRESS))
    return fail(SL_EINVAL, "unknown flag bits");
  if (o->strategy != SL_OMEGA_FIXED && o->strategy != SL_OMEGA_SCHEDULE && o->strategy != SL_OMEGA_ENUM &&
      o->strategy != SL_OMEGA_AUTO)
    return fail(SL_EINVAL, "unknown relaxation strategy %d", o->strategy);
  if (o->iter_offset < 0 || o->iter_offset > (int64_t)INT32_MAX * 64)
    return fail(SL_EINVAL, "iter_offset = %lld outside [0, 2^37]", (long long)o->iter_offset);
  if (o->strategy == SL_OMEGA_SCHEDULE) {
    if (!o->omega_schedule && o->max_iter > 0) return fail(SL_EINVAL, "SL_OMEGA_SCHEDULE needs omega_schedule");
    for (int64_t g = o->iter_offset; g < o->iter_offset + o->max_iter; ++g)
      if (!(std::isfinite(o->omega_schedule[g]) && o->omega_schedule[g] > 0.0 && o->omega_schedule[g] <= 16.0))
        return fail(SL_EINVAL, "omega_schedule[%lld] = %g outside (0, 16]", (long long)g, o->omega_schedule[g]);
  } else if (o->omega_schedule) {
    return fail(SL_EINVAL, "omega_schedule is only read with SL_OMEGA_SCHEDULE");
  }
  if (o->omega_vertex && o->strategy != SL_OMEGA_FIXED)
    return fail(SL_EINVAL, "per-vertex factors need SL_OMEGA_FIXED");
  if (o->seed != 0 && o->strategy != SL_OMEGA_AUTO)
    return fail(SL_EINVAL, "seed is only read with SL_OMEGA_AUTO");
  if (o->ordering != SL_ORDER_JACOBI && o->ordering != SL_ORDER_EXACT)
    return fail(SL_EINVAL, "unknown ordering %d", o->ordering);
  if (!(std::isfinite(o->inner_tol) && o->inner_tol >= 0.0 && o->inner_tol < 1.0))
    return fail(SL_EINVAL, "inner_tol = %g outside [0, 1)", o->inner_tol);
  if (o->inner_max_iter < 0) return fail(SL_EINVAL, "inner_max_iter = %d is negative", o->inner_max_iter);
  return SL_OK;
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }

}  // namespace

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
struct sl_plan {
  int n = 0, n_pad = 0, dim = 2, vec = 2;
  Split sp{};
  hipStream_t ps = nullptr;     // the plan's own stream (default priority)
  hipEvent_t ev_a = nullptr, ev_b = nullptr, ev_sync = nullptr;
  uint8_t* d = nullptr;         // n_pad^2 bytes, tile-major (hop counts)
  // weighted graphs: FP32 distances instead of d, the shortest-path trees and
  // the CSR on the device (lengths can be replaced: sl_plan_set_lengths)
  float* df = nullptr;          // n_pad^2 floats, tile-major
  int32_t* pred = nullptr;      // n x n, row-major
  int64_t* g_row_ptr = nullptr;
  int32_t* g_col_idx = nullptr;
  float* g_len = nullptr;
  int32_t* g_erow = nullptr;    // source row of every CSR entry
  int64_t nnz = 0;
  // tape of the last sl_plan_unroll: checkpoints X^{m c} and the trace rows
  // (decisions) of every iteration; reverse-mode work buffers
  int tape_K = -1, tape_c = 1, tape_safeguard = 1, tape_sym = 0;
  double tape_omega = 1.0;
  float* ckpt = nullptr;
  size_t ckpt_cap = 0;          // floats
  double* tape_trace = nullptr;
  int tape_cap = 0;             // rows
  float* segX = nullptr;
  int seg_cap = 0;              // iterates
  double* gb = nullptr;         // 3 x n_pad adjoint of the iterate
  float* gvec = nullptr;        // per iteration of a segment: stride floats each
  float* wbar = nullptr;        // per iteration of a segment: n_pad floats each
  size_t gvec_cap = 0, wbar_cap = 0;  // floats allocated
  float* Dbar = nullptr;        // n_pad^2 (edge-length plans)
  float* Sbuf = nullptr;        // n x n (edge-length plans)
  double* Gedge = nullptr;      // nnz
  // force pass over unordered pairs (hop-count plans)
  int4* sym_items = nullptr;
  int32_t* sym_panel_items = nullptr;
  int nsym_items = 0;
  float* Pi = nullptr;          // row partials: items x sym_rows_per_item() x dim
  float* Pj = nullptr;          // column partials: panels x n_pad x dim
  double* edot = nullptr;       // unordered fused pass: per reduction workgroup, sum e_i . F_i(X~)
  double* W = nullptr;          // n_pad
  float* Xb = nullptr;          // 3 iterate buffers
  float* Eb = nullptr;          // x~ - x^H, same format as one iterate buffer
  size_t stride = 0;            // floats per iterate buffer
  double* fpart = nullptr;      // slices x 3 x n_pad
  double* spart = nullptr;      // slices x n_pad
  double* red = nullptr;        // nred x 8
  int nred = 0;
  double* sgpart = nullptr;     // one double per safeguard work item
  int4* items = nullptr;        // safeguard work items
  double* sched = nullptr;      // device copy of a relaxation schedule (paper's factors)
  int sched_cap = 0;
  int nsg = 0;
  DevState* st = nullptr;       // loop state
  DevState* st_eval = nullptr;  // state for stand-alone stress passes
  DevState* host_st = nullptr;  // pinned mirror
  int32_t* host_flags = nullptr;  // pinned: the level flags of the breadth-first sweeps
  double plan_ms = 0.0;
  // captured chunk of iterations, rebuilt when the loop parameters change
  hipGraphExec_t gexec = nullptr;
  std::vector<double> gkey;
  // exact step (allocated on first use)
  int32_t* comp = nullptr;      // lowest vertex of each vertex's component
  CgVectors cg{};               // y, r, z (columns) and p (per vertex), double
  LwSym lw_sym{};               // the L^W matvec over unordered pairs: work items and FP64 partials
  double* cg_part = nullptr;    // (kCgSlots x cg_blocks(n_pad) + matvec blocks) x 8
  CgState* cg_st = nullptr;
  CgState* host_cg = nullptr;   // pinned mirror
  hipGraphExec_t cg_gexec = nullptr;  // a group of conjugate-gradient steps
  std::vector<double> cg_gkey;
};

namespace {

sl_status free_plan_memory(sl_plan* p) {
  (void)hipFree(p->d);
  (void)hipFree(p->df);
  (void)hipFree(p->pred);
  (void)hipFree(p->g_row_ptr);
  (void)hipFree(p->g_col_idx);
  (void)hipFree(p->g_len);
  (void)hipFree(p->g_erow);
  (void)hipFree(p->ckpt);
  (void)hipFree(p->tape_trace);
  (void)hipFree(p->segX);
  (void)hipFree(p->gb);
  (void)hipFree(p->gvec);
  (void)hipFree(p->wbar);
  (void)hipFree(p->Dbar);
  (void)hipFree(p->Sbuf);
  (void)hipFree(p->Gedge);
  (void)hipFree(p->lw_sym.Pi);
  (void)hipFree(p->lw_sym.Pj);
  (void)hipFree(p->sym_items);
  (void)hipFree(p->sym_panel_items);
  (void)hipFree(p->Pi);
  (void)hipFree(p->Pj);
  (void)hipFree(p->edot);
  (void)hipFree(p->W);
  (void)hipFree(p->Xb);
  (void)hipFree(p->Eb);
  (void)hipFree(p->items);
  (void)hipFree(p->sched);
  (void)hipFree(p->fpart);
  (void)hipFree(p->spart);
  (void)hipFree(p->red);
  (void)hipFree(p->sgpart);
  (void)hipFree(p->st);
  (void)hipFree(p->st_eval);
  if (p->host_st) (void)hipHostFree(p->host_st);
  if (p->host_flags) (void)hipHostFree(p->host_flags);
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  (void)hipFree(p->comp);
  (void)hipFree(p->cg.y);
  (void)hipFree(p->cg.pd);
  (void)hipFree(p->cg_part);
  (void)hipFree(p->cg_st);
  if (p->host_cg) (void)hipHostFree(p->host_cg);
  if (p->cg_gexec) (void)hipGraphExecDestroy(p->cg_gexec);
  if (p->ev_a) (void)hipEventDestroy(p->ev_a);
  if (p->ev_b) (void)hipEventDestroy(p->ev_b);
  if (p->ev_sync) (void)hipEventDestroy(p->ev_sync);
  if (p->ps) (void)hipStreamDestroy(p->ps);
  return SL_OK;
}

sl_status join_from_stream(hipStream_t ps, hipEvent_t ev, hipStream_t user) {
  HIP_TRY(hipEventRecord(ev, user), "hipEventRecord");
  HIP_TRY(hipStreamWaitEvent(ps, ev, 0), "hipStreamWaitEvent");
  return SL_OK;
}

sl_status join_to_stream(hipStream_t ps, hipEvent_t ev, hipStream_t user) {
  HIP_TRY(hipEventRecord(ev, ps), "hipEventRecord");
  HIP_TRY(hipStreamWaitEvent(user, ev, 0), "hipStreamWaitEvent");
  return SL_OK;
}

sl_status hip_try_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  return SL_OK;
}

// Order the plan stream after the caller's stream.
sl_status join_from(sl_plan* p, hipStream_t user) {
  HIP_TRY(hipEventRecord(p->ev_sync, user), "hipEventRecord");
  HIP_TRY(hipStreamWaitEvent(p->ps, p->ev_sync, 0), "hipStreamWaitEvent");
  return SL_OK;
}

sl_status join_to(sl_plan* p, hipStream_t user) {
  HIP_TRY(hipEventRecord(p->ev_sync, p->ps), "hipEventRecord");
  HIP_TRY(hipStreamWaitEvent(user, p->ev_sync, 0), "hipStreamWaitEvent");
  return SL_OK;
}

// Level kBfsMaxLevel of the search only detects a distance beyond the 255 hops
// a byte holds.
constexpr int kBfsMaxLevel = 256;

// Multi-source BFS, bfs_sources_per_sweep() sources per sweep, then W.
// Distances above 255 hops are refused (SL_ERANGE).
// Weighted graphs: shortest paths on the device from the plan's CSR copy.
sl_status build_weighted(sl_plan* p) {
  HIP_TRY(hipMemsetAsync(p->df, 0, sizeof(float) * (size_t)p->n_pad * p->n_pad, p->ps), "hipMemsetAsync(d)");
  HIP_TRY(launch_wsssp(p->g_erow, p->g_col_idx, p->g_len, p->nnz, p->n, p->sp.ng, p->df, p->pred, p->ps),
          "shortest-path kernel");
  HIP_TRY(launch_wsym(p->df, p->n_pad, p->sp.ng, p->ps), "symmetrize kernel");
  HIP_TRY(launch_weights(nullptr, p->df, p->W, p->fpart, p->sp, p->n, p->ps), "weights kernel");
  return SL_OK;
}

sl_status build_distances(sl_plan* p, const sl_graph* g) {
  const int n = p->n;
  if (p->df) return build_weighted(p);
  if (n > 1 && g->nnz > 0) {
    if (g->nnz > (int64_t)INT32_MAX) return fail(SL_ERANGE, "more than 2^31 - 1 CSR entries");
    // The gather's runs (whole rows of at most bfs_run_entries() entries packed
    // together) and the rows that take a wave or a workgroup each (longer ones,
    // and isolated vertices), packed on a host thread of their own while this
    // one allocates the buffers (sized for at most n of each) and sends the CSR.
    std::vector<int4> runs;
    std::vector<int4> longrows;
    const int run_max = bfs_run_entries(), mid_max = bfs_mid_max_degree();
    int nbig = 0;
    auto pack = [&]() {
      int4 open_run = make_int4(0, 0, 0, 0);
      for (int v = 0; v < n; ++v) {
        const int64_t b0 = g->row_ptr[v], deg = g->row_ptr[v + 1] - b0;
        if (deg == 0 || deg > run_max) {
          longrows.push_back(make_int4(v, (int)b0, (int)deg, 0));
          if (deg > 0 && open_run.y > 0) {  // a run holds consecutive CSR entries: close it before this row's
            runs.push_back(open_run);
            open_run.y = 0;
          }
        } else {
          if (open_run.y > 0 && open_run.y + deg > run_max) {
            runs.push_back(open_run);
            open_run.y = 0;
          }
          if (open_run.y == 0) open_run = make_int4((int)b0, 0, v, 0);
          open_run.y += (int)deg;
        }
      }
      if (open_run.y > 0) runs.push_back(open_run);
      // the rows above the middle degree first (a workgroup each), then the others (a wave each)
      std::stable_partition(longrows.begin(), longrows.end(), [&](const int4& r) { return r.z > mid_max; });
      nbig = (int)std::count_if(longrows.begin(), longrows.end(), [&](const int4& r) { return r.z > mid_max; });
    };
    bool packed = true;  // false: a host container could not grow
    auto pack_here = [&]() {
      try {
        pack();
      } catch (...) {
        packed = false;
      }
    };
    std::thread packer;
    try {
      packer = std::thread(pack_here);
    } catch (...) {
      pack_here();  // no thread to be had: pack on this one
    }
    auto join = [&]() {
      if (packer.joinable()) packer.join();
    };
    const size_t words = (size_t)n * bfs_words();
    const int nslots = bfs_slots();
    const int sweep = bfs_sources_per_sweep();
    const int nsweeps = (n + sweep - 1) / sweep;
    constexpr int kStride = kBfsMaxLevel + 1;  // one flag row per sweep: flags[l], l = 0 .. 256
    // one device allocation for the search's buffers, 256-byte aligned parts
    size_t off = 0;
    auto part = [&](size_t bytes) {
      const size_t at = off;
      off += (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
      return at;
    };
    const size_t o_ci = part(sizeof(int32_t) * g->nnz), o_rp = part(sizeof(int64_t) * (n + 1)),
                 o_rn = part(sizeof(int4) * n), o_pairs = part(sizeof(int2) * (size_t)n * run_max),
                 o_lrows = part(sizeof(int4) * n), o_slots = part(sizeof(uint64_t) * words * nslots),
                 o_masks = part(sizeof(uint64_t) * (size_t)n * nslots),
                 o_flag = part(sizeof(int32_t) * kStride * nsweeps),
                 o_wq = part(sizeof(double) * (size_t)bfs_weight_partials() * p->n_pad);
    char* buf = nullptr;
    sl_status status = SL_OK;
    auto cleanup = [&]() {
      (void)hipStreamSynchronize(p->ps);
      (void)hipFree(buf);
    };
    hipError_t e = hipMalloc(&buf, off);
    if (e != hipSuccess) {
      join();
      return hip_fail(e, "distance buffers");
    }
    int32_t* ci = reinterpret_cast<int32_t*>(buf + o_ci);
    int64_t* rp = reinterpret_cast<int64_t*>(buf + o_rp);
    int4* rn = reinterpret_cast<int4*>(buf + o_rn);
    int2* pairs = reinterpret_cast<int2*>(buf + o_pairs);
    int4* lrows = reinterpret_cast<int4*>(buf + o_lrows);
    uint64_t* slots = reinterpret_cast<uint64_t*>(buf + o_slots);
    uint64_t* masks = reinterpret_cast<uint64_t*>(buf + o_masks);
    int32_t* flag = reinterpret_cast<int32_t*>(buf + o_flag);
    double* wq = reinterpret_cast<double*>(buf + o_wq);
    int32_t* hflag = p->host_flags;
    e = hipMemcpyAsync(ci, g->col_idx, sizeof(int32_t) * g->nnz, hipMemcpyHostToDevice, p->ps);
    if (e == hipSuccess) e = hipMemcpyAsync(rp, g->row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, p->ps);
    join();
    if (!packed) {
      cleanup();
      return fail(SL_ENOMEM, "host allocation failed (the search's runs)");
    }
    const int nruns = (int)runs.size();
    const int nmid = (int)longrows.size() - nbig;
    if (e == hipSuccess && nruns > 0)
      e = hipMemcpyAsync(rn, runs.data(), sizeof(int4) * nruns, hipMemcpyHostToDevice, p->ps);
    if (e == hipSuccess && !longrows.empty())
      e = hipMemcpyAsync(lrows, longrows.data(), sizeof(int4) * longrows.size(), hipMemcpyHostToDevice, p->ps);
    if (e == hipSuccess) e = launch_bfs_pairs(rn, nruns, rp, ci, pairs, p->ps);
    if (e == hipSuccess) e = hipMemsetAsync(wq, 0, sizeof(double) * (size_t)bfs_weight_partials() * p->n_pad, p->ps);
    if (e == hipSuccess) e = launch_bfs_flags(flag, nsweeps, kStride, p->ps);
    if (e != hipSuccess) {
      cleanup();
      return hip_fail(e, "distance buffers");
    }
    // Every byte of d is written by the first batch of levels of some sweep
    // (the sweeps' column ranges cover [0, n_pad), and every row is stored).
    // Levels l0 .. l1 of sweep sw (one batch, at most nslots levels), then their distances.
    auto queue_levels = [&](int sw, int l0, int l1, int count_from) -> hipError_t {
      int32_t* fl = flag + (size_t)sw * kStride;
      hipError_t le = hipSuccess;
      for (int level = l0; level <= l1 && le == hipSuccess; ++level)
        le = launch_bfs_level(pairs, nruns, lrows, nbig, nmid, ci, slots, masks, n, sw * sweep, level, fl, p->ps);
      // level 256 is not stored: it only tells whether a distance exceeds 255
      if (le == hipSuccess)
        le = launch_bfs_store(slots, masks, fl, p->d, wq, n, p->n_pad, sw * sweep, l0, std::min(l1, kBfsMaxLevel - 1),
                              count_from, p->ps);
      return le;
    };
    // A sweep run batch by batch, the host reading the batch's flags after each
    // one, until its search ends (its depth) or passes 255 hops.  Levels below
    // count_from are not counted again (a sweep redone after a shorter run).
    auto sweep_synced = [&](int sw, int first_batch, int count_from, int* depth) -> hipError_t {
      int32_t* fl = flag + (size_t)sw * kStride;
      hipError_t le = launch_bfs_flags(fl, 1, kStride, p->ps);
      for (int l0 = 1, l1 = 0; le == hipSuccess; l0 = l1 + 1) {
        l1 = std::min(l0 + (l0 == 1 ? first_batch : nslots) - 1, kBfsMaxLevel);
        le = queue_levels(sw, l0, l1, count_from);
        if (le == hipSuccess)
          le = hipMemcpyAsync(hflag, fl + l0, sizeof(int32_t) * (l1 - l0 + 1), hipMemcpyDeviceToHost, p->ps);
        if (le == hipSuccess) le = hipStreamSynchronize(p->ps);
        if (le != hipSuccess) break;
        if (hflag[l1 - l0] == 0) {  // the search ended in this batch
          *depth = l0 - 1;
          for (int l = l0; l <= l1 && hflag[l - l0]; ++l) *depth = l;
          break;
        }
        if (l1 == kBfsMaxLevel) {
          status = fail(SL_ERANGE, "a graph distance exceeds 255 hops (sources %d..%d)", sw * sweep,
                        sw * sweep + sweep - 1);
          break;
        }
      }
      return le;
    };
    // The first sweep learns the search depth D.  The others are queued back
    // to back with D + 2 levels each and no host wait; a sweep whose level
    // D + 2 still found something is redone batch by batch afterwards.
    int depth = 0;
    e = sweep_synced(0, nslots, 1, &depth);
    const int L = std::min(depth + 2, kBfsMaxLevel);
    for (int sw = 1; sw < nsweeps && e == hipSuccess && status == SL_OK; ++sw)
      for (int l0 = 1; l0 <= L && e == hipSuccess; l0 += nslots) e = queue_levels(sw, l0, std::min(l0 + nslots - 1, L), 1);
    if (e == hipSuccess && status == SL_OK && nsweeps > 1) {
      e = hipMemcpyAsync(hflag, flag, sizeof(int32_t) * kStride * nsweeps, hipMemcpyDeviceToHost, p->ps);
      if (e == hipSuccess) e = hipStreamSynchronize(p->ps);
      for (int sw = 1; sw < nsweeps && e == hipSuccess && status == SL_OK; ++sw) {
        if (!hflag[(size_t)sw * kStride + L]) continue;
        // levels 1 .. L of this sweep are in d and the weights; find the rest
        int dsw = 0;
        e = sweep_synced(sw, nslots, L + 1, &dsw);
      }
    }
    if (e == hipSuccess && status == SL_OK) e = launch_weights_from_partials(wq, p->W, n, p->n_pad, p->ps);
    cleanup();
    if (e != hipSuccess) return hip_fail(e, "breadth-first search");
    return status;
  }
  HIP_TRY(hipMemsetAsync(p->d, 0, (size_t)p->n_pad * p->n_pad, p->ps), "hipMemsetAsync(d)");
  HIP_TRY(launch_weights(p->d, nullptr, p->W, p->fpart, p->sp, n, p->ps), "weights kernel");
  return SL_OK;
}

// The steps of one iteration after X^H is known (or, for the Jacobi step, after
// the force pass): update + extrapolation, safeguard or enumeration, select,
// and the optional position trace.
sl_status enqueue_after_force(sl_plan* p, const LoopParams& lp, const sl_options* o) {
  HIP_TRY(launch_update(p->dim, lp, p->fpart, p->spart, p->W, p->Xb, p->stride, p->Eb, p->st, p->red, p->ps),
          "update kernel");
  if (lp.enumerate)
    HIP_TRY(launch_sgdelta_enum(p->dim, p->d, p->Xb, p->stride, p->Eb, p->items, p->nsg, p->st, p->sgpart, p->sp,
                                p->ps),
            "enumeration kernel");
  else if (lp.safeguard && (lp.omega_p != 0.0 || lp.omega_sched || lp.omega_vertex))
    HIP_TRY(launch_sgdelta(p->dim, p->d, p->df, p->Xb, p->stride, p->Eb, p->items, p->nsg, p->st, p->sgpart, p->sp,
                           p->ps),
            "safeguard kernel");
  HIP_TRY(launch_select(p->dim, lp, p->red, p->nred, p->sgpart, p->nsg, p->st, o->trace, p->ps), "select kernel");
  if (lp.enumerate)
    HIP_TRY(launch_apply_enum(p->Eb, p->Xb, p->stride, p->st, p->n, p->dim, p->ps), "enumeration apply kernel");
  if (o->xtrace) HIP_TRY(launch_record(p->Xb, p->stride, p->st, o->xtrace, p->n, p->dim, p->ps), "record kernel");
  return SL_OK;
}

// Buffers of the unordered-pair force pass, made on first use: its work items
// and the row and column partial sums.
// The force pass taken by default: once per unordered pair where that is the
// faster one, else every ordered pair (measured in 2-D and 3-D, BA graphs):
//   hop counts     n_pad >= kSymMinN; from kSymMinNFused in a run whose passes
//                  carry the safeguard (their bounds cost far less than the
//                  difference the ordered pass sums)
//   edge lengths   n_pad >= kSymMinNLengths (the ordered pass reads 4-byte
//                  distances twice)
constexpr int kSymMinN = 24576;
constexpr int kSymMinNFused = 16384;
constexpr int kSymMinNLengths = 16384;
bool sym_by_default(const sl_plan* p, bool fused) {
  if (p->n <= 1) return false;
  if (p->df) return p->n_pad >= kSymMinNLengths;
  return p->n_pad >= (fused ? kSymMinNFused : kSymMinN);
}

sl_status ensure_sym(sl_plan* p) {
  if (p->sym_items) return SL_OK;
  if (p->n <= 1) return fail(SL_ENOTSUP, "the unordered-pair force pass needs n > 1");
  const SymSplit ss = make_sym_split(p->n_pad);
  int4* items = nullptr;
  int32_t* panel_items = nullptr;
  float* Pi = nullptr;
  float* Pj = nullptr;
  double* edot = nullptr;
  hipError_t e = hipMalloc(&items, sizeof(int4) * ss.items.size());
  if (e == hipSuccess) e = hipMalloc(&edot, sizeof(double) * sym_reduce_blocks(p->n_pad));
  if (e == hipSuccess) e = hipMalloc(&panel_items, sizeof(int32_t) * ss.panel_items.size());
  if (e == hipSuccess) e = hipMalloc(&Pi, sizeof(float) * ss.items.size() * sym_rows_per_item() * p->dim);
  if (e == hipSuccess) e = hipMalloc(&Pj, sizeof(float) * (size_t)ss.npanels * p->n_pad * p->dim);
  if (e == hipSuccess)
    e = hipMemcpyAsync(items, ss.items.data(), sizeof(int4) * ss.items.size(), hipMemcpyHostToDevice, p->ps);
  if (e == hipSuccess)
    e = hipMemcpyAsync(panel_items, ss.panel_items.data(), sizeof(int32_t) * ss.panel_items.size(),
                       hipMemcpyHostToDevice, p->ps);
  if (e == hipSuccess) e = hipStreamSynchronize(p->ps);  // the split's host vectors are temporaries
  if (e != hipSuccess) {
    (void)hipFree(items);
    (void)hipFree(panel_items);
    (void)hipFree(Pi);
    (void)hipFree(Pj);
    (void)hipFree(edot);
    return hip_fail(e, "unordered-pair force pass setup");
  }
  p->edot = edot;
  p->sym_items = items;
  p->sym_panel_items = panel_items;
  p->Pi = Pi;
  p->Pj = Pj;
  p->nsym_items = (int)ss.items.size();
  return SL_OK;
}

sl_status enqueue_force(sl_plan* p, const LoopParams& lp) {
  if (lp.sym) {
    HIP_TRY(launch_force_sym(p->dim, 0, p->d, p->df, p->Xb, p->stride, p->st, p->sym_items, p->nsym_items,
                             p->sym_panel_items, p->Pi, p->Pj, p->fpart, p->n_pad, p->ps),
            "symmetric force kernels");
    return SL_OK;
  }
  HIP_TRY(launch_force(p->dim, lp.stress != 0, p->d, p->df, p->Xb, p->stride, p->st, p->fpart, p->spart, p->sp, p->n_pad,
                       p->ps),
          "force kernel");
  return SL_OK;
}

// The step tail with the safeguard in the next force pass: the update (X^H,
// X~), the force at X~ with f(X~) - f(X^H) summed in, the decision, and the
// force at X^H when X~ lost.  fpart then holds the force at X^{k+1}.
sl_status enqueue_fused_tail(sl_plan* p, const LoopParams& lp, const sl_options* o) {
  HIP_TRY(launch_update(p->dim, lp, p->fpart, p->spart, p->W, p->Xb, p->stride, p->Eb, p->st, p->red, p->ps),
          "update kernel");
  if (lp.sym) {
    // the pass at X~ with the bounds U >= f(X~) - f(X^H) >= L; the exact
    // difference (and its select) only when they leave its sign open
    // (the exact variant instead after an iteration whose bounds left it open,
    // until they would have decided again: both launches are gated by the state)
    // (one of the two runs in each iteration: one reduction after both)
    for (int exact = 0; exact < 2; ++exact)
      HIP_TRY(launch_force_sym_sg(p->dim, lp, exact, 1, exact ? kSymReduceAny : kSymReduceNone, p->d, p->df, p->Xb,
                                  p->stride, p->Eb, p->st, p->sym_items,
                                  p->nsym_items, p->sym_panel_items, p->Pi, p->Pj, p->sgpart, p->fpart, p->edot,
                                  p->n_pad, p->ps),
              "symmetric fused force and safeguard kernels");
    HIP_TRY(launch_select(p->dim, lp, p->red, p->nred, p->sgpart, p->nsym_items, p->st, o->trace, p->ps,
                          kSelectBounds, p->edot, (int)sym_reduce_blocks(p->n_pad)),
            "select kernel");
    HIP_TRY(launch_sgdelta(p->dim, p->d, p->df, p->Xb, p->stride, p->Eb, p->items, p->nsg, p->st, p->sgpart, p->sp,
                           p->ps, 1),
            "safeguard kernel");
    HIP_TRY(launch_select(p->dim, lp, p->red, p->nred, p->sgpart, p->nsg, p->st, o->trace, p->ps, kSelectExact),
            "select kernel");
    HIP_TRY(launch_force_sym(p->dim, 1, p->d, p->df, p->Xb, p->stride, p->st, p->sym_items, p->nsym_items,
                             p->sym_panel_items, p->Pi, p->Pj, p->fpart, p->n_pad, p->ps),
            "symmetric force kernels");
  } else {
    HIP_TRY(launch_force_sg(p->dim, lp, p->d, p->df, p->Xb, p->stride, p->Eb, p->st, p->fpart, p->sgpart, p->sp,
                            p->ps),
            "fused force and safeguard kernel");
    HIP_TRY(launch_select(p->dim, lp, p->red, p->nred, p->sgpart, p->sp.blocks_x * p->sp.slices, p->st, o->trace,
                          p->ps),
            "select kernel");
    HIP_TRY(launch_force_cond(p->dim, p->d, p->df, p->Xb, p->stride, p->st, p->fpart, p->sp, p->n_pad, p->ps),
            "force kernel");
  }
  if (o->xtrace) HIP_TRY(launch_record(p->Xb, p->stride, p->st, o->xtrace, p->n, p->dim, p->ps), "record kernel");
  return SL_OK;
}

sl_status enqueue_iteration(sl_plan* p, const LoopParams& lp, const sl_options* o) {
  // fused: the force of X^k came from the previous iteration (or the pass before the loop)
  if (lp.fuse) return enqueue_fused_tail(p, lp, o);
  sl_status s = enqueue_force(p, lp);
  if (s != SL_OK) return s;
  return enqueue_after_force(p, lp, o);
}

// Buffers of the exact step and the component of every vertex.
sl_status ensure_exact(sl_plan* p) {
  if (p->cg_st) return SL_OK;
  const size_t col = (size_t)3 * p->n_pad;
  const size_t nrec = (size_t)kCgSlots * cg_blocks(p->n_pad) +
                      std::max<size_t>((size_t)p->sp.blocks_x * p->sp.slices, lw_sym_reduce_blocks(p->n_pad));
  hipError_t e = hipMalloc(&p->comp, sizeof(int32_t) * p->n_pad);
  if (e == hipSuccess) e = hipMalloc(&p->cg.y, sizeof(double) * 3 * col);
  if (e == hipSuccess) e = hipMalloc(&p->cg.pd, sizeof(double) * p->stride);
  if (e == hipSuccess) e = hipMalloc(&p->cg_part, sizeof(double) * nrec * 8);
  if (e == hipSuccess) e = hipHostMalloc(&p->host_cg, sizeof(CgState), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc(&p->cg_st, sizeof(CgState));
  if (e != hipSuccess) {
    (void)hipFree(p->cg_st);
    p->cg_st = nullptr;
    return hip_fail(e, "exact-step buffers");
  }
  p->cg.n_pad = p->n_pad;
  p->cg.r = p->cg.y + col;
  p->cg.z = p->cg.y + 2 * col;
  HIP_TRY(hipMemsetAsync(p->cg.y, 0, sizeof(double) * 3 * col, p->ps), "hipMemsetAsync");
  HIP_TRY(hipMemsetAsync(p->cg.pd, 0, sizeof(double) * p->stride, p->ps), "hipMemsetAsync");
  HIP_TRY(hipMemsetAsync(p->cg_part, 0, sizeof(double) * nrec * 8, p->ps), "hipMemsetAsync");
  HIP_TRY(hipMemsetAsync(p->cg_st, 0, sizeof(CgState), p->ps), "hipMemsetAsync");
  HIP_TRY(launch_components(p->d, p->comp, p->n, p->n_pad, p->sp.ng, p->ps), "components kernel");
  return SL_OK;
}

// The exact step's L^W matvec over unordered pairs (hop-count plans): by
// default in 2-D from n_pad = kLwSymMinN, where reading d once per unordered
// pair pays for the column reductions; SL_FLAG_SYM_FORCE / SL_FLAG_ORDERED_FORCE
// choose.
constexpr int kLwSymMinN = 24576;
bool lw_sym_for(const sl_plan* p, uint32_t flags) {
  if (p->n <= 1 || p->df) return false;
  if (flags & SL_FLAG_SYM_FORCE) return true;
  if (flags & SL_FLAG_ORDERED_FORCE) return false;
  return p->dim == 2 && p->n_pad >= kLwSymMinN;
}

// Its FP64 partial sums (and the force pass's work items), made on first use.
sl_status ensure_lw_sym(sl_plan* p) {
  if (p->lw_sym.Pi) return SL_OK;
  sl_status s = ensure_sym(p);
  if (s != SL_OK) return s;
  const int rows = sym_rows_per_item();
  const size_t npanels = ((size_t)p->n_pad + rows - 1) / rows;
  double *Pi = nullptr, *Pj = nullptr;
  hipError_t e = hipMalloc(&Pi, sizeof(double) * (size_t)p->nsym_items * rows * p->dim);
  if (e == hipSuccess) e = hipMalloc(&Pj, sizeof(double) * npanels * p->n_pad * p->dim);
  if (e != hipSuccess) {
    (void)hipFree(Pi);
    (void)hipFree(Pj);
    return hip_fail(e, "unordered-pair matvec buffers");
  }
  p->lw_sym.items = p->sym_items;
  p->lw_sym.nitems = p->nsym_items;
  p->lw_sym.panel_items = p->sym_panel_items;
  p->lw_sym.Pi = Pi;
  p->lw_sym.Pj = Pj;
  return SL_OK;
}

constexpr int kCgGroup = 8;  // conjugate-gradient steps per launch between host polls

sl_status enqueue_cg_group(sl_plan* p, double itol, int imax, bool lws) {
  for (int k = 0; k < kCgGroup; ++k)
    HIP_TRY(launch_cg_step(p->dim, p->cg, p->d, p->W, p->comp, p->n, p->st, p->cg_st, p->cg_part, p->fpart, p->sp,
                           itol, imax, lws ? &p->lw_sym : nullptr, p->ps),
            "conjugate-gradient kernels");
  return SL_OK;
}

// Algorithm 2 with the exact step: per iteration the force pass (r_0), the
// solve in groups of kCgGroup steps until its stop flag, then the common tail.
// With lp.fuse the force at X^k comes from the previous iteration's fused tail
// (or the pass before the loop).
sl_status run_exact(sl_plan* p, LoopParams lp, const sl_options* o, bool use_graph, int* inner_total) {
  sl_status s = ensure_exact(p);
  if (s != SL_OK) return s;
  const bool lws = lw_sym_for(p, o->flags);
  if (lws && (s = ensure_lw_sym(p)) != SL_OK) return s;
  lp.exact_y = p->cg.y;
  const double itol = o->inner_tol > 0.0 ? o->inner_tol : 1e-6;
  const int imax = o->inner_max_iter > 0 ? o->inner_max_iter : 500;
  if (use_graph) {
    const std::vector<double> key = {(double)p->dim, itol, (double)imax, lws ? 1.0 : 0.0};
    if (!p->cg_gexec || key != p->cg_gkey) {
      if (p->cg_gexec) {
        (void)hipGraphExecDestroy(p->cg_gexec);
        p->cg_gexec = nullptr;
      }
      hipGraph_t graph = nullptr;
      HIP_TRY(hipStreamBeginCapture(p->ps, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
      const sl_status cs = enqueue_cg_group(p, itol, imax, lws);
      const hipError_t ce = hipStreamEndCapture(p->ps, &graph);
      if (cs != SL_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return cs;
      }
      if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
      const hipError_t ie = hipGraphInstantiate(&p->cg_gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) {
        p->cg_gexec = nullptr;
        return hip_fail(ie, "hipGraphInstantiate");
      }
      p->cg_gkey = key;
    }
  }
  DevState* h = p->host_st;
  CgState* hc = p->host_cg;
  const int max_groups = imax / kCgGroup + 2;
  *inner_total = 0;
  for (int k = 0; k < o->max_iter && !h->done; ++k) {
    if (!lp.fuse && (s = enqueue_force(p, lp)) != SL_OK) return s;
    HIP_TRY(launch_cg_init(p->dim, p->cg, p->fpart, p->sp.slices, p->W, p->comp, p->n, p->Xb, p->stride, p->st, p->cg_st,
                           p->cg_part, p->ps),
            "conjugate-gradient init kernel");
    bool stopped = false;
    for (int G = 0; G < max_groups && !stopped; ++G) {
      if (use_graph) HIP_TRY(hipGraphLaunch(p->cg_gexec, p->ps), "hipGraphLaunch");
      else if ((s = enqueue_cg_group(p, itol, imax, lws)) != SL_OK) return s;
      HIP_TRY(hipMemcpyAsync(hc, p->cg_st, sizeof(CgState), hipMemcpyDeviceToHost, p->ps), "solver state download");
      HIP_TRY(hipStreamSynchronize(p->ps), "hipStreamSynchronize");
      stopped = hc->done != 0;
    }
    if (!stopped) return fail(SL_EDEVICE, "the conjugate-gradient solve did not reach its stop flag");
    *inner_total += hc->iters;
    if ((s = lp.fuse ? enqueue_fused_tail(p, lp, o) : enqueue_after_force(p, lp, o)) != SL_OK) return s;
    HIP_TRY(hipMemcpyAsync(h, p->st, sizeof(DevState), hipMemcpyDeviceToHost, p->ps), "state download");
    HIP_TRY(hipStreamSynchronize(p->ps), "hipStreamSynchronize");
  }
  return SL_OK;
}

sl_status stress_pass(sl_plan* p, int cur, double* f) {
  DevState* h = p->host_st;
  std::memset(h, 0, sizeof(DevState));
  h->cur = cur;
  HIP_TRY(hipMemcpyAsync(p->st_eval, h, sizeof(DevState), hipMemcpyHostToDevice, p->ps), "state upload");
  HIP_TRY(launch_force(p->dim, true, p->d, p->df, p->Xb, p->stride, p->st_eval, p->fpart, p->spart, p->sp, p->n_pad,
                       p->ps),
          "force kernel");
  HIP_TRY(launch_stress_sum(p->spart, p->sp.slices, p->n_pad, p->st_eval, p->ps), "stress kernel");
  HIP_TRY(hipMemcpyAsync(h, p->st_eval, sizeof(DevState), hipMemcpyDeviceToHost, p->ps), "state download");
  HIP_TRY(hipStreamSynchronize(p->ps), "hipStreamSynchronize");
  *f = h->stress;
  return SL_OK;
}

// The probabilistic strategy's draw of iteration g (Sec. 5.2): output number g
// (from 0) of SplitMix64 seeded with `seed` (Steele, Lea and Flood, OOPSLA 2014),
// as a uniform u = (z >> 11) 2^-53 in [0, 1), through the roulette over the
// paper's factors 0.5, 1.0, 1.5, 2.0 with probabilities 0.3, 0.3, 0.2, 0.2.
double auto_factor(uint64_t seed, uint64_t g) {
  uint64_t z = seed + (g + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const double u = (double)(z >> 11) * 0x1.0p-53;
  return u < 0.3 ? 0.5 : (u < 0.6 ? 1.0 : (u < 0.8 ? 1.5 : 2.0));
}

// The paper's factors of iterations iter_offset .. iter_offset + max_iter - 1
// (a caller's schedule, or the probabilistic strategy's draws) into the plan's
// device array, indexed by the iteration of the call.
sl_status upload_schedule(sl_plan* p, const sl_options* o) {
  if (p->sched_cap < o->max_iter) {
    (void)hipFree(p->sched);
    p->sched = nullptr;
    p->sched_cap = 0;
    HIP_TRY(hipMalloc(&p->sched, sizeof(double) * o->max_iter), "schedule buffer");
    p->sched_cap = o->max_iter;
    if (p->gexec) {  // the captured iterations read the old array
      (void)hipGraphExecDestroy(p->gexec);
      p->gexec = nullptr;
    }
  }
  std::vector<double> wp(o->max_iter);
  for (int k = 0; k < o->max_iter; ++k) {
    const int64_t g = o->iter_offset + k;
    wp[k] = o->strategy == SL_OMEGA_AUTO ? auto_factor(o->seed, (uint64_t)g) : o->omega_schedule[g] - 1.0;
  }
  HIP_TRY(hipMemcpyAsync(p->sched, wp.data(), sizeof(double) * o->max_iter, hipMemcpyHostToDevice, p->ps),
          "schedule upload");
  HIP_TRY(hipStreamSynchronize(p->ps), "hipStreamSynchronize");  // wp is a host temporary
  return SL_OK;
}

// f of the returned placement (eq. 1) and the relative stress decrease of the
// last iteration, (f(X^{K-1}) - f(X^K)) / f(X^{K-1}), the reading of the
// paper's "rel err" (Table 1); NaN with SL_FLAG_NO_FINAL_STRESS.
sl_status final_stress(sl_plan* p, const DevState& fin, uint32_t flags, sl_result* res) {
  res->stress = std::nan("");
  res->rel_stress_drop = std::nan("");
  if (flags & SL_FLAG_NO_FINAL_STRESS) return SL_OK;
  double f = 0.0;
  sl_status s;
  if (p->n > 1 && (s = stress_pass(p, fin.cur, &f)) != SL_OK) return s;
  res->stress = f;
  if (p->n > 1 && fin.iter > 0 && fin.status == 0) {  // X^{K-1} is intact after a completed iteration
    double fp = 0.0;
    if ((s = stress_pass(p, fin.prev, &fp)) != SL_OK) return s;
    if (fp != 0.0) res->rel_stress_drop = (fp - f) / fp;
  }
  return SL_OK;
}

}  // namespace

extern "C" {

void sl_default_options(sl_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->dim = 2;
  o->max_iter = 1000;
  o->omega = 1.0;
  o->tol = 1e-3;
  o->safeguard = 1;
}

const char* sl_last_error(void) { return g_err.c_str(); }

sl_status sl_validate(const sl_graph* g, const sl_options* opt) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    sl_status s = check_graph(g);
    if (s != SL_OK) return s;
    if (opt) return check_options(opt);
    return SL_OK;
  });
}

sl_status sl_plan_create(const sl_graph* g, int32_t dim, void* stream, sl_plan** out) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    if (!out) return fail(SL_EINVAL, "out is NULL");
    *out = nullptr;
    sl_status s = check_graph(g);
    if (s != SL_OK) return s;
    if (dim != 2 && dim != 3) return fail(SL_EINVAL, "dim = %d, expected 2 or 3", dim);
    sl_plan* p = new (std::nothrow) sl_plan();
    if (!p) return fail(SL_ENOMEM, "host allocation failed");
    p->n = g->n;
    p->n_pad = std::max(64, round_up(g->n, 64));
    p->dim = dim;
    p->vec = dim == 2 ? 2 : 4;
    p->sp = make_split(p->n_pad);
    p->stride = (size_t)p->n_pad * p->vec;
    p->nred = (p->n_pad + 255) / 256;
    const std::vector<int4> items = triangle_items(p->sp);
    p->nsg = (int)items.size();
    hipStream_t user = (hipStream_t)stream;
    auto bail = [&](sl_status st) {
      free_plan_memory(p);
      delete p;
      return st;
    };
    hipError_t e = hipStreamCreateWithFlags(&p->ps, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&p->ev_a);
    if (e == hipSuccess) e = hipEventCreate(&p->ev_b);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_sync, hipEventDisableTiming);
    if (g->edge_len) {
      p->nnz = g->nnz;
      if (e == hipSuccess) e = hipMalloc(&p->df, sizeof(float) * (size_t)p->n_pad * p->n_pad);
      if (e == hipSuccess) e = hipMalloc(&p->pred, sizeof(int32_t) * std::max<size_t>(1, (size_t)p->n * p->n));
      if (e == hipSuccess) e = hipMalloc(&p->g_row_ptr, sizeof(int64_t) * (p->n + 1));
      if (e == hipSuccess) e = hipMalloc(&p->g_col_idx, sizeof(int32_t) * std::max<int64_t>(1, g->nnz));
      if (e == hipSuccess) e = hipMalloc(&p->g_len, sizeof(float) * std::max<int64_t>(1, g->nnz));
      if (e == hipSuccess)
        e = hipMemcpyAsync(p->g_row_ptr, g->row_ptr, sizeof(int64_t) * (p->n + 1), hipMemcpyHostToDevice, p->ps);
      if (e == hipSuccess && g->nnz > 0)
        e = hipMemcpyAsync(p->g_col_idx, g->col_idx, sizeof(int32_t) * g->nnz, hipMemcpyHostToDevice, p->ps);
      if (e == hipSuccess && g->nnz > 0)
        e = hipMemcpyAsync(p->g_len, g->edge_len, sizeof(float) * g->nnz, hipMemcpyHostToDevice, p->ps);
      std::vector<int32_t> erow((size_t)g->nnz);
      for (int v = 0; v < g->n; ++v)
        for (int64_t q = g->row_ptr[v]; q < g->row_ptr[v + 1]; ++q) erow[(size_t)q] = v;
      if (e == hipSuccess) e = hipMalloc(&p->g_erow, sizeof(int32_t) * std::max<int64_t>(1, g->nnz));
      if (e == hipSuccess && g->nnz > 0)
        e = hipMemcpyAsync(p->g_erow, erow.data(), sizeof(int32_t) * g->nnz, hipMemcpyHostToDevice, p->ps);
      if (e == hipSuccess) e = hipStreamSynchronize(p->ps);  // erow is a host temporary
    } else if (e == hipSuccess) {
      e = hipMalloc(&p->d, (size_t)p->n_pad * p->n_pad);
    }
    if (e == hipSuccess) e = hipMalloc(&p->W, sizeof(double) * p->n_pad);
    if (e == hipSuccess) e = hipMalloc(&p->Xb, sizeof(float) * 3 * p->stride);
    if (e == hipSuccess) e = hipMalloc(&p->Eb, sizeof(float) * p->stride);
    if (e == hipSuccess) e = hipMalloc(&p->items, sizeof(int4) * items.size());
    if (e == hipSuccess) e = hipMalloc(&p->fpart, sizeof(double) * p->sp.slices * 3 * p->n_pad);
    if (e == hipSuccess) e = hipMalloc(&p->spart, sizeof(double) * p->sp.slices * p->n_pad);
    if (e == hipSuccess) e = hipMalloc(&p->red, sizeof(double) * 8 * p->nred);
    if (e == hipSuccess)
      e = hipMalloc(&p->sgpart, sizeof(double) * std::max<size_t>({(size_t)p->nsg * kEnumCandidates,
                                                                   (size_t)p->sp.blocks_x * p->sp.slices,
                                                                   3 * make_sym_split(p->n_pad).items.size()}));
    if (e == hipSuccess) e = hipMalloc(&p->st, sizeof(DevState));
    if (e == hipSuccess) e = hipMalloc(&p->st_eval, sizeof(DevState));
    if (e == hipSuccess) e = hipHostMalloc(&p->host_st, sizeof(DevState), hipHostMallocDefault);
    if (e == hipSuccess && !g->edge_len && g->n > 1 && g->nnz > 0) {
      const size_t sweeps = ((size_t)g->n + bfs_sources_per_sweep() - 1) / bfs_sources_per_sweep();
      e = hipHostMalloc(&p->host_flags, sizeof(int32_t) * (kBfsMaxLevel + 1) * sweeps, hipHostMallocDefault);
    }
    if (e != hipSuccess) return bail(hip_fail(e, "plan allocation"));
    e = hipMemsetAsync(p->Xb, 0, sizeof(float) * 3 * p->stride, p->ps);
    if (e == hipSuccess) e = hipMemsetAsync(p->Eb, 0, sizeof(float) * p->stride, p->ps);
    if (e == hipSuccess)
      e = hipMemcpyAsync(p->items, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice, p->ps);
    if (e != hipSuccess) return bail(hip_fail(e, "plan initialization"));
    if ((s = join_from(p, user)) != SL_OK) return bail(s);
    if ((e = hipEventRecord(p->ev_a, p->ps)) != hipSuccess) return bail(hip_fail(e, "hipEventRecord"));
    if ((s = build_distances(p, g)) != SL_OK) return bail(s);
    if ((e = hipEventRecord(p->ev_b, p->ps)) != hipSuccess) return bail(hip_fail(e, "hipEventRecord"));
    if ((e = hipStreamSynchronize(p->ps)) != hipSuccess) return bail(hip_fail(e, "hipStreamSynchronize"));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p->ev_a, p->ev_b);
    p->plan_ms = ms;
    *out = p;
    return SL_OK;
  });
}

sl_status sl_plan_destroy(sl_plan* p) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    if (!p) return SL_OK;
    (void)hipStreamSynchronize(p->ps);
    free_plan_memory(p);
    delete p;
    return SL_OK;
  });
}

sl_status sl_plan_run(sl_plan* p, float* X, const sl_options* o, void* stream, sl_result* out) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    if (!p) return fail(SL_EINVAL, "plan is NULL");
    sl_status s = check_options(o);
    if (s != SL_OK) return s;
    if (o->dim != p->dim) return fail(SL_EINVAL, "options dim %d differs from the plan's %d", o->dim, p->dim);
    if (!X && p->n > 0) return fail(SL_EINVAL, "X is NULL");
    if (p->df && (o->strategy == SL_OMEGA_ENUM || o->ordering == SL_ORDER_EXACT))
      return fail(SL_ENOTSUP, "edge-length plans run the Jacobi step with a fixed, scheduled or per-vertex factor");
    hipStream_t user = (hipStream_t)stream;
    sl_result res{};
    res.plan_ms = p->plan_ms;
    LoopParams lp{};
    lp.n = p->n;
    lp.n_pad = p->n_pad;
    lp.ng = p->sp.ng;
    lp.nrb = p->sp.nrb;
    lp.slices = p->sp.slices;
    lp.groups_per_slice = p->sp.groups_per_slice;
    lp.omega_p = o->omega - 1.0;
    lp.tol = o->tol;
    lp.safeguard = o->safeguard;
    lp.stress = (o->flags & SL_FLAG_TRACE_STRESS) ? 1 : 0;
    lp.enumerate = o->strategy == SL_OMEGA_ENUM ? 1 : 0;
    lp.omega_vertex = o->omega_vertex;
    lp.omega_sched = nullptr;
    // the safeguard rides on the next force pass: a safeguard to evaluate, no
    // enumeration or stress trace
    lp.fuse = (lp.safeguard && !lp.enumerate && !lp.stress &&
               !(o->flags & SL_FLAG_SEPARATE_SAFEGUARD) &&
               (lp.omega_p != 0.0 || o->strategy == SL_OMEGA_SCHEDULE || o->strategy == SL_OMEGA_AUTO ||
                o->omega_vertex) &&
               p->n > 1)
                  ? 1
                  : 0;
    if ((o->flags & SL_FLAG_SYM_FORCE) && (o->flags & SL_FLAG_ORDERED_FORCE))
      return fail(SL_EINVAL, "SL_FLAG_SYM_FORCE and SL_FLAG_ORDERED_FORCE exclude each other");
    // with the exact step the flag chooses the L^W matvec (run_exact); the force pass stays ordered
    lp.sym = (o->flags & SL_FLAG_SYM_FORCE) && o->ordering == SL_ORDER_JACOBI ? 1 : 0;
    if ((o->flags & SL_FLAG_SYM_FORCE) && lp.stress) return fail(SL_ENOTSUP, "SL_FLAG_SYM_FORCE: no stress trace");
    if (!(o->flags & SL_FLAG_ORDERED_FORCE) && !lp.stress && o->ordering == SL_ORDER_JACOBI &&
        sym_by_default(p, lp.fuse != 0))
      lp.sym = 1;
    if (lp.sym) {
      if (p->n > 1 && (s = ensure_sym(p)) != SL_OK) return s;
      if (p->n <= 1) lp.sym = 0;
      else lp.slices = 1;
    }

    if ((s = join_from(p, user)) != SL_OK) return s;
    if (o->omega_vertex && p->n > 0) {
      std::vector<float> wv(p->n);
      HIP_TRY(hipMemcpyAsync(wv.data(), o->omega_vertex, sizeof(float) * p->n, hipMemcpyDeviceToHost, p->ps),
              "omega_vertex copy");
      HIP_TRY(hipStreamSynchronize(p->ps), "hipStreamSynchronize");
      for (int i = 0; i < p->n; ++i)
        if (!(std::isfinite(wv[i]) && wv[i] > 0.f && wv[i] <= 16.f))
          return fail(SL_EINVAL, "omega_vertex[%d] = %g outside (0, 16]", i, (double)wv[i]);
    }
    if ((o->strategy == SL_OMEGA_SCHEDULE || o->strategy == SL_OMEGA_AUTO) && o->max_iter > 0) {
      if ((s = upload_schedule(p, o)) != SL_OK) return s;
      lp.omega_sched = p->sched;
    }
    if (p->n > 0) HIP_TRY(launch_pack_in(X, p->Xb, p->n, p->n_pad, p->dim, p->ps), "pack kernel");
    DevState* h = p->host_st;
    std::memset(h, 0, sizeof(DevState));
    h->max_iter = o->max_iter;
    h->done = (o->max_iter == 0 || p->n <= 1) ? 1 : 0;
    h->converged = p->n <= 1 ? 1 : 0;
    HIP_TRY(hipMemcpyAsync(p->st, h, sizeof(DevState), hipMemcpyHostToDevice, p->ps), "state upload");

    // iterations per captured graph between looks at the stop flag (those after
    // the stop return at once)
    // (not capped by max_iter: runs of any length replay the same captured graph,
    // whose iterations after the stop return at once)
    const int chunk = o->check_every > 0 ? o->check_every : (p->n <= 8192 ? 32 : 8);
    const bool use_graph = !(o->flags & SL_FLAG_NO_GRAPH);
    const bool exact = o->ordering == SL_ORDER_EXACT;
    if (use_graph && !exact) {
      std::vector<double> key = {(double)p->dim, lp.omega_p, lp.tol, (double)lp.safeguard, (double)lp.stress,
                                 (double)lp.sym, (double)lp.fuse,
                                 (double)chunk, (double)(uintptr_t)o->trace, (double)(uintptr_t)o->xtrace,
                                 (double)lp.enumerate, (double)(uintptr_t)lp.omega_sched,
                                 (double)(uintptr_t)lp.omega_vertex};
      if (!p->gexec || key != p->gkey) {
        if (p->gexec) {
          (void)hipGraphExecDestroy(p->gexec);
          p->gexec = nullptr;
        }
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(p->ps, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        sl_status cs = SL_OK;
        for (int k = 0; k < chunk && cs == SL_OK; ++k) cs = enqueue_iteration(p, lp, o);
        hipError_t ce = hipStreamEndCapture(p->ps, &graph);
        if (cs != SL_OK) {
          if (graph) (void)hipGraphDestroy(graph);
          return cs;
        }
        if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
        hipError_t ie = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
          p->gexec = nullptr;
          return hip_fail(ie, "hipGraphInstantiate");
        }
        p->gkey = key;
      }
    }
    HIP_TRY(hipEventRecord(p->ev_a, p->ps), "hipEventRecord");
    if (lp.fuse && (s = enqueue_force(p, lp)) != SL_OK) return s;  // the force at X^0
    if (exact) {
      int inner = 0;
      if ((s = run_exact(p, lp, o, use_graph, &inner)) != SL_OK) return s;
      res.inner_iterations = inner;
    }
    const int max_launches = exact ? 0 : o->max_iter / chunk + 2;
    for (int L = 0; L < max_launches; ++L) {
      if (use_graph) {
        HIP_TRY(hipGraphLaunch(p->gexec, p->ps), "hipGraphLaunch");
      } else {
        for (int k = 0; k < chunk; ++k)
          if ((s = enqueue_iteration(p, lp, o)) != SL_OK) return s;
      }
      HIP_TRY(hipMemcpyAsync(h, p->st, sizeof(DevState), hipMemcpyDeviceToHost, p->ps), "state download");
      HIP_TRY(hipStreamSynchronize(p->ps), "hipStreamSynchronize");
      if (h->done) break;
    }
    HIP_TRY(hipEventRecord(p->ev_b, p->ps), "hipEventRecord");
    HIP_TRY(hipEventSynchronize(p->ev_b), "hipEventSynchronize");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p->ev_a, p->ev_b);
    res.run_ms = ms;
    const DevState fin = *h;
    if (!fin.done) return fail(SL_EDEVICE, "iteration loop did not reach its stop flag");
    if (p->n > 0) HIP_TRY(launch_pack_out(p->Xb, p->st, p->stride, X, p->n, p->dim, p->ps), "unpack kernel");
    res.iterations = fin.iter;
    res.converged = fin.converged;
    res.rejected = fin.rejected;
    res.residual = fin.residual;
    if ((s = final_stress(p, fin, o->flags, &res)) != SL_OK) return s;
    if ((s = join_to(p, user)) != SL_OK) return s;
    if (out) *out = res;
    if (fin.status != 0)
      return fail(SL_ENUMERIC, "non-finite coordinate at iteration %d; X holds the last finite iterate", fin.iter + 1);
    return SL_OK;
  });
}

sl_status sl_plan_stress(sl_plan* p, const float* X, int32_t dim, void* stream, double* f) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    if (!p || !f) return fail(SL_EINVAL, "plan or f is NULL");
    if (dim != p->dim) return fail(SL_EINVAL, "dim %d differs from the plan's %d", dim, p->dim);
    if (!X && p->n > 0) return fail(SL_EINVAL, "X is NULL");
    sl_status s = join_from(p, (hipStream_t)stream);
    if (s != SL_OK) return s;
    if (p->n <= 1) {
      *f = 0.0;
      return SL_OK;
    }
    HIP_TRY(launch_pack_in(X, p->Xb, p->n, p->n_pad, p->dim, p->ps), "pack kernel");
    if ((s = stress_pass(p, 0, f)) != SL_OK) return s;
    return join_to(p, (hipStream_t)stream);
  });
}

sl_status sl_plan_profile(sl_plan* p, const float* X, int32_t dim, double omega, int32_t reps, void* stream,
                          double* ms) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    if (!p || !ms) return fail(SL_EINVAL, "plan or ms is NULL");
    if (dim != p->dim) return fail(SL_EINVAL, "dim %d differs from the plan's %d", dim, p->dim);
    if (!X && p->n > 0) return fail(SL_EINVAL, "X is NULL");
    if (reps < 1) return fail(SL_EINVAL, "reps must be >= 1");
    if (!(std::isfinite(omega) && omega > 0.0 && omega <= 16.0)) return fail(SL_EINVAL, "omega outside (0, 16]");
    sl_status s = join_from(p, (hipStream_t)stream);
    if (s != SL_OK) return s;
    for (int k = 0; k < 9; ++k) ms[k] = 0.0;
    if (p->n <= 1) return SL_OK;
    if (!p->df && (s = ensure_exact(p)) != SL_OK) return s;  // the L^W matvec exists for hop-count plans
    const bool lws = lw_sym_for(p, 0);  // the exact step's default matvec
    if (lws && (s = ensure_lw_sym(p)) != SL_OK) return s;
    LoopParams lp{};
    lp.n = p->n;
    lp.n_pad = p->n_pad;
    lp.ng = p->sp.ng;
    lp.nrb = p->sp.nrb;
    lp.slices = p->sp.slices;
    lp.groups_per_slice = p->sp.groups_per_slice;
    lp.omega_p = omega - 1.0;
    lp.tol = -1.0;  // never stop while timing
    lp.safeguard = 1;
    lp.stress = 0;
    lp.sym = 0;  // the force pass sl_plan_run uses by default
    if ((s = ensure_sym(p)) != SL_OK) return s;  // for ms[5] and ms[7]
    HIP_TRY(launch_pack_in(X, p->Xb, p->n, p->n_pad, p->dim, p->ps), "pack kernel");
    DevState* h = p->host_st;
    std::memset(h, 0, sizeof(DevState));
    h->max_iter = INT32_MAX;
    HIP_TRY(hipMemcpyAsync(p->st, h, sizeof(DevState), hipMemcpyHostToDevice, p->ps), "state upload");
    LoopParams lpf = lp;  // the fused pass, extrapolating with omega
    lpf.fuse = 1;
    lpf.safeguard = 1;
    for (int which = 0; which < 9; ++which) {
      if (which == 4 && p->df) continue;
      if (which == 4) {  // a solver state from the current placement: r_0, z
        HIP_TRY(launch_force(p->dim, false, p->d, p->df, p->Xb, p->stride, p->st, p->fpart, p->spart, p->sp, p->n_pad,
                             p->ps), "force kernel");
        HIP_TRY(launch_cg_init(p->dim, p->cg, p->fpart, p->sp.slices, p->W, p->comp, p->n, p->Xb, p->stride, p->st, p->cg_st,
                               p->cg_part, p->ps),
                "conjugate-gradient init kernel");
      }
      for (int r = -1; r < reps; ++r) {  // one untimed launch first
        if (r == 0) HIP_TRY(hipEventRecord(p->ev_a, p->ps), "hipEventRecord");
        switch (which) {
          case 4:
            if (lws)
              HIP_TRY(launch_lw_sym(p->dim, p->cg.pd, p->d, p->W, p->st, p->cg_st, p->lw_sym, p->fpart,
                                    p->cg_part + (size_t)kCgSlots * cg_blocks(p->n_pad) * 8, p->n_pad, p->ps),
                      "L^W kernels");
            else
              HIP_TRY(launch_lw(p->dim, p->cg, p->d, p->W, p->st, p->cg_st, p->fpart,
                                p->cg_part + (size_t)kCgSlots * cg_blocks(p->n_pad) * 8, p->sp, p->ps),
                      "L^W kernel");
            break;
          case 0:
            if ((s = enqueue_force(p, lp)) != SL_OK) return s;
            break;
          case 6:
            HIP_TRY(launch_force_sg(p->dim, lpf, p->d, p->df, p->Xb, p->stride, p->Eb, p->st, p->fpart, p->sgpart,
                                    p->sp, p->ps),
                    "fused force and safeguard kernel");
            break;
          case 5:
            HIP_TRY(launch_force_sym(p->dim, 0, p->d, p->df, p->Xb, p->stride, p->st, p->sym_items, p->nsym_items,
                                     p->sym_panel_items, p->Pi, p->Pj, p->fpart, p->n_pad, p->ps),
                    "symmetric force kernels");
            break;
          case 7:
            HIP_TRY(launch_force_sym_sg(p->dim, lpf, 0, 0, kSymReducePass, p->d, p->df, p->Xb, p->stride, p->Eb, p->st,
                                        p->sym_items,
                                        p->nsym_items, p->sym_panel_items, p->Pi, p->Pj, p->sgpart, p->fpart, p->edot,
                                        p->n_pad, p->ps),
                    "symmetric fused force and safeguard kernels");
            break;
          case 8:
            HIP_TRY(launch_force_sym_sg(p->dim, lpf, 1, 0, kSymReducePass, p->d, p->df, p->Xb, p->stride, p->Eb, p->st,
                                        p->sym_items,
                                        p->nsym_items, p->sym_panel_items, p->Pi, p->Pj, p->sgpart, p->fpart, p->edot,
                                        p->n_pad, p->ps),
                    "symmetric fused force and exact safeguard kernels");
            break;
          case 1:
            HIP_TRY(launch_update(p->dim, lp, p->fpart, p->spart, p->W, p->Xb, p->stride, p->Eb, p->st, p->red,
                                  p->ps),
                    "update kernel");
            break;
          case 2:
            HIP_TRY(launch_sgdelta(p->dim, p->d, p->df, p->Xb, p->stride, p->Eb, p->items, p->nsg, p->st, p->sgpart,
                                   p->sp, p->ps),
                    "safeguard kernel");
            break;
          default:
            HIP_TRY(launch_select(p->dim, lp, p->red, p->nred, p->sgpart, p->nsg, p->st, nullptr, p->ps),
                    "select kernel");
        }
      }
      HIP_TRY(hipEventRecord(p->ev_b, p->ps), "hipEventRecord");
      HIP_TRY(hipEventSynchronize(p->ev_b), "hipEventSynchronize");
      float t = 0.f;
      HIP_TRY(hipEventElapsedTime(&t, p->ev_a, p->ev_b), "hipEventElapsedTime");
      ms[which] = (double)t / reps;
    }
    return join_to(p, (hipStream_t)stream);
  });
}

namespace {

sl_status check_rows(const sl_plan* p, const int32_t* rows, int32_t nrows, const void* out) {
  if (!p) return fail(SL_EINVAL, "plan is NULL");
  if (nrows < 0) return fail(SL_EINVAL, "nrows is negative");
  if (nrows > 0 && (!rows || !out)) return fail(SL_EINVAL, "rows or out is NULL");
  for (int k = 0; k < nrows; ++k)
    if (rows[k] < 0 || rows[k] >= p->n) return fail(SL_EINVAL, "row %d outside [0, n)", rows[k]);
  return SL_OK;
}

// Distances of the listed rows as floats (hop counts or lengths) into host out.
sl_status gather_rows(sl_plan* p, const int32_t* rows, int32_t nrows, hipStream_t stream, float* out) {
  sl_status s = join_from(p, stream);
  if (s != SL_OK) return s;
  int32_t* drows = nullptr;
  float* dout = nullptr;
  const size_t count = (size_t)nrows * p->n;
  hipError_t e = hipMalloc(&drows, sizeof(int32_t) * nrows);
  if (e == hipSuccess) e = hipMalloc(&dout, sizeof(float) * count);
  if (e == hipSuccess) e = hipMemcpyAsync(drows, rows, sizeof(int32_t) * nrows, hipMemcpyHostToDevice, p->ps);
  if (e == hipSuccess) e = launch_gather_rows(p->d, p->df, drows, nrows, p->n, p->sp.ng, dout, p->ps);
  if (e == hipSuccess) e = hipMemcpyAsync(out, dout, sizeof(float) * count, hipMemcpyDeviceToHost, p->ps);
  if (e == hipSuccess) e = hipStreamSynchronize(p->ps);
  (void)hipFree(drows);
  (void)hipFree(dout);
  if (e != hipSuccess) return hip_fail(e, "distance rows");
  return SL_OK;
}

}  // namespace

sl_status sl_plan_distance_rows(sl_plan* p, const int32_t* rows, int32_t nrows, void* stream, uint8_t* out) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    sl_status s = check_rows(p, rows, nrows, out);
    if (s != SL_OK) return s;
    if (p->df) return fail(SL_EINVAL, "the plan holds edge-length distances: use sl_plan_distance_rows_f32");
    if (nrows == 0 || p->n == 0) return SL_OK;
    std::vector<float> tmp((size_t)nrows * p->n);
    if ((s = gather_rows(p, rows, nrows, (hipStream_t)stream, tmp.data())) != SL_OK) return s;
    for (size_t q = 0; q < tmp.size(); ++q) out[q] = (uint8_t)tmp[q];
    return SL_OK;
  });
}

sl_status sl_plan_distance_rows_f32(sl_plan* p, const int32_t* rows, int32_t nrows, void* stream, float* out) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    sl_status s = check_rows(p, rows, nrows, out);
    if (s != SL_OK) return s;
    if (nrows == 0 || p->n == 0) return SL_OK;
    return gather_rows(p, rows, nrows, (hipStream_t)stream, out);
  });
}

sl_status sl_plan_tree_rows(sl_plan* p, const int32_t* rows, int32_t nrows, void* stream, int32_t* out) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    sl_status s = check_rows(p, rows, nrows, out);
    if (s != SL_OK) return s;
    if (!p->pred) return fail(SL_EINVAL, "shortest-path trees are kept for edge-length plans only");
    if (nrows == 0 || p->n == 0) return SL_OK;
    if ((s = join_from(p, (hipStream_t)stream)) != SL_OK) return s;
    for (int k = 0; k < nrows; ++k)
      HIP_TRY(hipMemcpyAsync(out + (size_t)k * p->n, p->pred + (size_t)rows[k] * p->n, sizeof(int32_t) * p->n,
                             hipMemcpyDeviceToHost, p->ps),
              "tree rows copy");
    HIP_TRY(hipStreamSynchronize(p->ps), "hipStreamSynchronize");
    return SL_OK;
  });
}

sl_status sl_plan_set_lengths(sl_plan* p, const float* edge_len, void* stream) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    if (!p) return fail(SL_EINVAL, "plan is NULL");
    if (!p->df) return fail(SL_EINVAL, "the plan was created without edge lengths");
    if (p->nnz > 0 && !edge_len) return fail(SL_EINVAL, "edge_len is NULL");
    std::vector<int64_t> rp(p->n + 1);
    std::vector<int32_t> ci((size_t)p->nnz);
    sl_status s = join_from(p, (hipStream_t)stream);
    if (s != SL_OK) return s;
    HIP_TRY(hipMemcpyAsync(rp.data(), p->g_row_ptr, sizeof(int64_t) * (p->n + 1), hipMemcpyDeviceToHost, p->ps),
            "graph copy");
    if (p->nnz > 0)
      HIP_TRY(hipMemcpyAsync(ci.data(), p->g_col_idx, sizeof(int32_t) * p->nnz, hipMemcpyDeviceToHost, p->ps),
              "graph copy");
    HIP_TRY(hipStreamSynchronize(p->ps), "hipStreamSynchronize");
    sl_graph g{p->n, p->nnz, rp.data(), ci.data(), edge_len};
    if ((s = check_lengths(&g, edge_len)) != SL_OK) return s;
    if (p->nnz > 0)
      HIP_TRY(hipMemcpyAsync(p->g_len, edge_len, sizeof(float) * p->nnz, hipMemcpyHostToDevice, p->ps),
              "lengths upload");
    HIP_TRY(hipEventRecord(p->ev_a, p->ps), "hipEventRecord");
    if ((s = build_weighted(p)) != SL_OK) return s;
    HIP_TRY(hipEventRecord(p->ev_b, p->ps), "hipEventRecord");
    HIP_TRY(hipStreamSynchronize(p->ps), "hipStreamSynchronize");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p->ev_a, p->ev_b);
    p->plan_ms = ms;
    return join_to(p, (hipStream_t)stream);
  });
}

sl_status sl_plan_weights(sl_plan* p, void* stream, double* W) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    if (!p || !W) return fail(SL_EINVAL, "plan or W is NULL");
    if (p->n == 0) return SL_OK;
    sl_status s = join_from(p, (hipStream_t)stream);
    if (s != SL_OK) return s;
    HIP_TRY(hipMemcpyAsync(W, p->W, sizeof(double) * p->n, hipMemcpyDeviceToHost, p->ps), "weights copy");
    HIP_TRY(hipStreamSynchronize(p->ps), "hipStreamSynchronize");
    return SL_OK;
  });
}

namespace {

sl_status grow(void** ptr, size_t* cap, size_t want, size_t elem, const char* what) {
  if (*cap >= want && *ptr) return SL_OK;
  (void)hipFree(*ptr);
  *ptr = nullptr;
  *cap = 0;
  HIP_TRY(hipMalloc(ptr, elem * std::max<size_t>(want, 1)), what);
  *cap = want;
  return SL_OK;
}

// The force pass an unrolled run takes: SL_FLAG_SYM_FORCE / SL_FLAG_ORDERED_FORCE
// as in sl_plan_run, else the default by size; SL_ENOTSUP where the unordered
// pass does not apply (n <= 1).
sl_status unroll_sym(sl_plan* p, uint32_t flags, bool fused, int* sym) {
  if ((flags & SL_FLAG_SYM_FORCE) && (flags & SL_FLAG_ORDERED_FORCE))
    return fail(SL_EINVAL, "SL_FLAG_SYM_FORCE and SL_FLAG_ORDERED_FORCE exclude each other");
  *sym = (flags & SL_FLAG_SYM_FORCE) ? 1 : (flags & SL_FLAG_ORDERED_FORCE) ? 0 : (sym_by_default(p, fused) ? 1 : 0);
  if (p->n <= 1) *sym = 0;
  if (*sym) return ensure_sym(p);
  return SL_OK;
}

LoopParams unroll_params(const sl_plan* p, double omega, int safeguard, int sym) {
  LoopParams lp{};
  lp.n = p->n;
  lp.n_pad = p->n_pad;
  lp.ng = p->sp.ng;
  lp.nrb = p->sp.nrb;
  lp.slices = p->sp.slices;
  lp.groups_per_slice = p->sp.groups_per_slice;
  lp.omega_p = omega - 1.0;
  lp.tol = -1.0;  // an unrolled run takes every one of its iterations
  lp.safeguard = safeguard;
  // the safeguard rides on the next force pass; a run (or a recomputed
  // segment) starts with one plain force pass
  lp.fuse = (safeguard && omega != 1.0 && p->n > 1) ? 1 : 0;
  // the force pass of the run (its buffers made by ensure_sym)
  if (sym) {
    lp.sym = 1;
    lp.slices = 1;
  }
  return lp;
}

// Upload a loop state: X^k in buffer 0, iteration k of max_iter.
sl_status set_state(sl_plan* p, DevState* dst, int iter, int max_iter) {
  DevState* h = p->host_st;
  std::memset(h, 0, sizeof(DevState));
  h->iter = iter;
  h->max_iter = max_iter;
  h->done = (iter >= max_iter || p->n <= 1) ? 1 : 0;
  h->converged = p->n <= 1 ? 1 : 0;
  HIP_TRY(hipMemcpyAsync(dst, h, sizeof(DevState), hipMemcpyHostToDevice, p->ps), "state upload");
  HIP_TRY(hipStreamSynchronize(p->ps), "hipStreamSynchronize");
  return SL_OK;
}

}  // namespace

sl_status sl_plan_stress_grad(sl_plan* p, const float* X, int32_t dim, void* stream, double* f, float* G) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    if (!p || !f) return fail(SL_EINVAL, "plan or f is NULL");
    if (dim != p->dim) return fail(SL_EINVAL, "dim %d differs from the plan's %d", dim, p->dim);
    if ((!X || !G) && p->n > 0) return fail(SL_EINVAL, "X or G is NULL");
    sl_status s = join_from(p, (hipStream_t)stream);
    if (s != SL_OK) return s;
    *f = 0.0;
    if (p->n == 0) return SL_OK;
    if (p->n == 1) {
      HIP_TRY(hipMemsetAsync(G, 0, sizeof(float) * dim, p->ps), "hipMemsetAsync");
      return join_to(p, (hipStream_t)stream);
    }
    HIP_TRY(launch_pack_in(X, p->Xb, p->n, p->n_pad, p->dim, p->ps), "pack kernel");
    if ((s = stress_pass(p, 0, f)) != SL_OK) return s;
    HIP_TRY(launch_stress_grad_out(p->fpart, p->sp.slices, p->n, p->n_pad, p->dim, G, p->ps), "gradient kernel");
    return join_to(p, (hipStream_t)stream);
  });
}

sl_status sl_plan_unroll(sl_plan* p, float* X, const sl_options* o, int32_t ckpt_every, void* stream,
                         sl_result* out) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    if (!p) return fail(SL_EINVAL, "plan is NULL");
    sl_status s = check_options(o);
    if (s != SL_OK) return s;
    if (o->dim != p->dim) return fail(SL_EINVAL, "options dim %d differs from the plan's %d", o->dim, p->dim);
    if (!X && p->n > 0) return fail(SL_EINVAL, "X is NULL");
    if (o->strategy != SL_OMEGA_FIXED || o->omega_vertex || o->ordering != SL_ORDER_JACOBI)
      return fail(SL_ENOTSUP, "unrolled runs take the Jacobi step with a fixed omega");
    if (o->trace || o->xtrace) return fail(SL_EINVAL, "unrolled runs keep their own trace");
    if (ckpt_every < 1) return fail(SL_EINVAL, "ckpt_every = %d must be >= 1", ckpt_every);
    const int K = o->max_iter, c = ckpt_every;
    const int nseg = (K + c - 1) / c;
    if ((s = join_from(p, (hipStream_t)stream)) != SL_OK) return s;
    size_t cap = p->ckpt_cap;
    if ((s = grow((void**)&p->ckpt, &cap, (size_t)std::max(nseg, 1) * p->stride, sizeof(float), "checkpoints")) != SL_OK)
      return s;
    p->ckpt_cap = cap;
    size_t tcap = (size_t)p->tape_cap * SL_TRACE_COLS;
    if ((s = grow((void**)&p->tape_trace, &tcap, (size_t)std::max(K, 1) * SL_TRACE_COLS, sizeof(double), "tape")) != SL_OK)
      return s;
    p->tape_cap = (int)(tcap / SL_TRACE_COLS);
    p->tape_K = -1;
    sl_options oo = *o;
    oo.trace = p->tape_trace;
    oo.xtrace = nullptr;
    oo.flags &= ~SL_FLAG_TRACE_STRESS;
    int sym = 0;
    // the rule of sl_plan_run, so that the unrolled run equals it bit for bit
    if ((s = unroll_sym(p, o->flags, o->safeguard && o->omega != 1.0 && p->n > 1, &sym)) != SL_OK) return s;
    const LoopParams lp = unroll_params(p, o->omega, o->safeguard, sym);
    sl_result res{};
    res.plan_ms = p->plan_ms;
    if (p->n > 0) HIP_TRY(launch_pack_in(X, p->Xb, p->n, p->n_pad, p->dim, p->ps), "pack kernel");
    if ((s = set_state(p, p->st, 0, K)) != SL_OK) return s;
    HIP_TRY(hipEventRecord(p->ev_a, p->ps), "hipEventRecord");
    if (K > 0) HIP_TRY(launch_save(p->Xb, p->stride, p->st, p->ckpt, p->ps), "checkpoint kernel");
    if (lp.fuse && K > 0 && (s = enqueue_force(p, lp)) != SL_OK) return s;  // the force at X^0
    for (int k = 0; k < K && p->n > 1; ++k) {
      if ((s = enqueue_iteration(p, lp, &oo)) != SL_OK) return s;
      if ((k + 1) % c == 0 && k + 1 < K)
        HIP_TRY(launch_save(p->Xb, p->stride, p->st, p->ckpt + (size_t)((k + 1) / c) * p->stride, p->ps),
                "checkpoint kernel");
    }
    HIP_TRY(hipEventRecord(p->ev_b, p->ps), "hipEventRecord");
    DevState* h = p->host_st;
    HIP_TRY(hipMemcpyAsync(h, p->st, sizeof(DevState), hipMemcpyDeviceToHost, p->ps), "state download");
    HIP_TRY(hipStreamSynchronize(p->ps), "hipStreamSynchronize");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p->ev_a, p->ev_b);
    res.run_ms = ms;
    const DevState fin = *h;
    if (p->n > 0) HIP_TRY(launch_pack_out(p->Xb, p->st, p->stride, X, p->n, p->dim, p->ps), "unpack kernel");
    res.iterations = fin.iter;
    res.converged = fin.converged;
    res.rejected = fin.rejected;
    res.residual = fin.residual;
    if ((s = final_stress(p, fin, o->flags, &res)) != SL_OK) return s;
    if ((s = join_to(p, (hipStream_t)stream)) != SL_OK) return s;
    if (out) *out = res;
    if (fin.status != 0)
      return fail(SL_ENUMERIC, "non-finite coordinate at iteration %d; X holds the last finite iterate", fin.iter + 1);
    p->tape_sym = sym;
    p->tape_K = K;
    p->tape_c = c;
    p->tape_omega = o->omega;
    p->tape_safeguard = o->safeguard;
    return SL_OK;
  });
}

sl_status sl_plan_unroll_backward(sl_plan* p, const float* G, float* gX0, float* glen, void* stream) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    if (!p) return fail(SL_EINVAL, "plan is NULL");
    if (p->tape_K < 0) return fail(SL_EINVAL, "no unrolled run to differentiate (call sl_plan_unroll first)");
    if ((!G || !gX0) && p->n > 0) return fail(SL_EINVAL, "G or gX0 is NULL");
    if (glen && !p->df) return fail(SL_EINVAL, "edge-length derivatives need a plan created with edge lengths");
    const int K = p->tape_K, c = p->tape_c;
    const int nseg = (K + c - 1) / c;
    sl_status s = join_from(p, (hipStream_t)stream);
    if (s != SL_OK) return s;
    if (p->n == 0) return SL_OK;
    const size_t col = (size_t)3 * p->n_pad;
    size_t cap = p->gb ? col : 0;
    if ((s = grow((void**)&p->gb, &cap, col, sizeof(double), "adjoint buffers")) != SL_OK) return s;
    if ((s = grow((void**)&p->gvec, &p->gvec_cap, (size_t)std::max(c, 1) * p->stride, sizeof(float),
                  "adjoint buffers")) != SL_OK)
      return s;
    if ((s = grow((void**)&p->wbar, &p->wbar_cap, (size_t)std::max(c, 1) * p->n_pad, sizeof(float),
                  "adjoint buffers")) != SL_OK)
      return s;
    size_t scap = (size_t)p->seg_cap * p->stride;
    if ((s = grow((void**)&p->segX, &scap, (size_t)std::max(c, 1) * p->stride, sizeof(float), "segment buffer")) != SL_OK)
      return s;
    p->seg_cap = (int)(scap / p->stride);
    if (glen) {
      cap = p->Dbar ? (size_t)p->n_pad * p->n_pad : 0;
      if ((s = grow((void**)&p->Dbar, &cap, (size_t)p->n_pad * p->n_pad, sizeof(float), "distance adjoint")) != SL_OK)
        return s;
      cap = p->Sbuf ? (size_t)p->n * p->n : 0;
      if ((s = grow((void**)&p->Sbuf, &cap, (size_t)p->n * p->n, sizeof(float), "distance adjoint")) != SL_OK) return s;
      cap = p->Gedge ? (size_t)p->nnz : 0;
      if ((s = grow((void**)&p->Gedge, &cap, (size_t)std::max<int64_t>(p->nnz, 1), sizeof(double), "edge adjoint")) !=
          SL_OK)
        return s;
      HIP_TRY(hipMemsetAsync(p->Dbar, 0, sizeof(float) * (size_t)p->n_pad * p->n_pad, p->ps), "hipMemsetAsync");
    }
    std::vector<double> tr((size_t)std::max(K, 1) * SL_TRACE_COLS);
    if (K > 0)
      HIP_TRY(hipMemcpyAsync(tr.data(), p->tape_trace, sizeof(double) * K * SL_TRACE_COLS, hipMemcpyDeviceToHost,
                             p->ps),
              "tape download");
    HIP_TRY(launch_grad_in(G, p->gb, p->n, p->n_pad, p->dim, p->ps), "gradient kernel");
    const LoopParams lp = unroll_params(p, p->tape_omega, p->tape_safeguard, p->tape_sym);
    sl_options oo;
    sl_default_options(&oo);
    oo.dim = p->dim;
    if ((s = set_state(p, p->st_eval, 0, 1)) != SL_OK) return s;  // cur = 0: force passes read the pointer given
    HIP_TRY(hipStreamSynchronize(p->ps), "hipStreamSynchronize");
    for (int m = nseg - 1; m >= 0 && p->n > 1; --m) {
      const int k0 = m * c, k1 = std::min(k0 + c, K);
      // recompute X^{k0} .. X^{k1-1} from the checkpoint
      HIP_TRY(hipMemcpyAsync(p->segX, p->ckpt + (size_t)m * p->stride, sizeof(float) * p->stride,
                             hipMemcpyDeviceToDevice, p->ps),
              "checkpoint copy");
      if (k1 - k0 > 1) {
        HIP_TRY(hipMemcpyAsync(p->Xb, p->segX, sizeof(float) * p->stride, hipMemcpyDeviceToDevice, p->ps),
                "checkpoint copy");
        if ((s = set_state(p, p->st, k0, K)) != SL_OK) return s;
        if (lp.fuse && (s = enqueue_force(p, lp)) != SL_OK) return s;  // the force at X^{k0}
        for (int q = 1; q < k1 - k0; ++q) {
          if ((s = enqueue_iteration(p, lp, &oo)) != SL_OK) return s;
          HIP_TRY(launch_save(p->Xb, p->stride, p->st, p->segX + (size_t)q * p->stride, p->ps), "save kernel");
        }
      }
      for (int k = k1 - 1; k >= k0; --k) {
        const float* Xk = p->segX + (size_t)(k - k0) * p->stride;
        // F at X^k by the pass the forward took (the unordered one leaves F in force slice 0)
        int fslices = p->sp.slices;
        if (lp.sym) {
          HIP_TRY(launch_force_sym(p->dim, 0, p->d, p->df, Xk, 0, p->st_eval, p->sym_items, p->nsym_items,
                                   p->sym_panel_items, p->Pi, p->Pj, p->fpart, p->n_pad, p->ps),
                  "force kernel");
          fslices = 1;
        } else {
          HIP_TRY(launch_force(p->dim, false, p->d, p->df, Xk, 0, p->st_eval, p->fpart, p->spart, p->sp, p->n_pad,
                               p->ps),
                  "force kernel");
        }
        const double a = tr[(size_t)k * SL_TRACE_COLS + 1] == 1.0 ? p->tape_omega : 1.0;
        HIP_TRY(launch_adjoint_step(p->dim, p->d, p->df, Xk, p->fpart, fslices, p->W, a, p->gb,
                                    p->gvec + (size_t)(k - k0) * p->stride, p->wbar + (size_t)(k - k0) * p->n_pad,
                                    p->fpart, p->sp, p->n_pad, p->ps),
                "adjoint kernels");
      }
      // dL/dd of the segment's iterations, added once per pair
      if (glen)
        HIP_TRY(launch_dbar_segment(p->dim, p->d, p->df, p->segX, p->stride, p->gvec, p->wbar, k1 - k0, p->Dbar, p->sp,
                                    p->n_pad, p->ps),
                "distance adjoint kernel");
    }
    HIP_TRY(launch_grad_out(p->gb, gX0, p->n, p->n_pad, p->dim, p->ps), "gradient kernel");
    if (glen) {
      HIP_TRY(launch_edge_grad(p->Dbar, p->Sbuf, p->g_row_ptr, p->g_col_idx, p->g_erow, p->pred, p->Gedge, glen,
                               p->n, p->nnz, p->n_pad, p->sp.ng, p->ps),
              "edge-length gradient kernels");
      if (p->n <= 1 || p->nnz == 0)
        HIP_TRY(hipMemsetAsync(glen, 0, sizeof(float) * std::max<int64_t>(p->nnz, 0), p->ps), "hipMemsetAsync");
    }
    HIP_TRY(hipStreamSynchronize(p->ps), "hipStreamSynchronize");
    return join_to(p, (hipStream_t)stream);
  });
}

sl_status sl_layout(const sl_graph* g, float* X, const sl_options* o, void* stream, sl_result* out) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    sl_status s = check_options(o);
    if (s != SL_OK) return s;
    sl_plan* p = nullptr;
    if ((s = sl_plan_create(g, o->dim, stream, &p)) != SL_OK) return s;
    s = sl_plan_run(p, X, o, stream, out);
    const ErrorText keep = g_err;
    sl_plan_destroy(p);
    g_err = keep;
    return s;
  });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched plans
// ---------------------------------------------------------------------------
struct sl_batch_plan {
  int ngraphs = 0, dim = 2, cus = 0, threads = 512;
  int64_t n_total = 0;
  hipStream_t ps = nullptr;
  hipEvent_t ev_a = nullptr, ev_b = nullptr, ev_sync = nullptr;
  std::vector<BatchGraph> hgraphs;
  std::vector<int32_t> horder;  // largest first
  BatchGraph* graphs = nullptr;
  int32_t* order = nullptr;
  int32_t* queue = nullptr;
  int32_t* status = nullptr;
  uint8_t* d = nullptr;
  double* W = nullptr;
  BatchResult* res = nullptr;
  std::vector<BatchResult> hres;
  double plan_ms = 0.0;
  hipGraphExec_t gexec = nullptr;
  std::vector<double> gkey;
};

namespace {

sl_status check_batch(const sl_batch* b) {
  if (!b) return fail(SL_EINVAL, "batch is NULL");
  if (b->num_graphs < 0) return fail(SL_EINVAL, "num_graphs is negative");
  if (b->num_graphs > 0 && !b->graph_ptr) return fail(SL_EINVAL, "graph_ptr is NULL");
  int64_t n_total = 0;
  if (b->num_graphs > 0) {
    if (b->graph_ptr[0] != 0) return fail(SL_EINVAL, "graph_ptr[0] must be 0");
    for (int g = 0; g < b->num_graphs; ++g) {
      const int64_t n = b->graph_ptr[g + 1] - b->graph_ptr[g];
      if (n < 0) return fail(SL_EINVAL, "graph_ptr decreases at graph %d", g);
      if (n > SL_BATCH_MAX_N) return fail(SL_EINVAL, "graph %d has %lld vertices, more than %d", g, (long long)n,
                                          SL_BATCH_MAX_N);
    }
    n_total = b->graph_ptr[b->num_graphs];
  }
  if (n_total > INT32_MAX) return fail(SL_EINVAL, "too many vertices in the batch");
  sl_graph g{};
  g.n = (int32_t)n_total;
  g.nnz = b->nnz;
  g.row_ptr = b->row_ptr;
  g.col_idx = b->col_idx;
  g.edge_len = nullptr;
  if (n_total == 0 && b->nnz != 0) return fail(SL_EINVAL, "empty batch with edges");
  sl_status s = check_graph(&g);
  if (s != SL_OK) return s;
  for (int gi = 0; gi < b->num_graphs; ++gi)
    for (int64_t v = b->graph_ptr[gi]; v < b->graph_ptr[gi + 1]; ++v)
      for (int64_t e = b->row_ptr[v]; e < b->row_ptr[v + 1]; ++e)
        if (b->col_idx[e] < b->graph_ptr[gi] || b->col_idx[e] >= b->graph_ptr[gi + 1])
          return fail(SL_EINVAL, "edge (%lld, %d) leaves graph %d", (long long)v, b->col_idx[e], gi);
  return SL_OK;
}

void free_batch(sl_batch_plan* p) {
  (void)hipFree(p->graphs);
  (void)hipFree(p->order);
  (void)hipFree(p->queue);
  (void)hipFree(p->status);
  (void)hipFree(p->d);
  (void)hipFree(p->W);
  (void)hipFree(p->res);
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->ev_a) (void)hipEventDestroy(p->ev_a);
  if (p->ev_b) (void)hipEventDestroy(p->ev_b);
  if (p->ev_sync) (void)hipEventDestroy(p->ev_sync);
  if (p->ps) (void)hipStreamDestroy(p->ps);
}

// Column slices that give every wave of a `threads` workgroup a unit, within
// the LDS budget of the force partials.
int default_slices(int n_pad, int threads) { return batch_default_slices(n_pad, threads); }

bool slices_ok(int n_pad, int s) { return s >= 1 && s <= n_pad / kColGroup && s * n_pad <= kBatchMaxPartial; }

int batch_blocks(const sl_batch_plan* p, int count) { return batch_layout_blocks(p->dim, p->cus, count); }

sl_status batch_upload_graphs(sl_batch_plan* p) {
  HIP_TRY(hipMemcpyAsync(p->graphs, p->hgraphs.data(), sizeof(BatchGraph) * p->hgraphs.size(),
                         hipMemcpyHostToDevice, p->ps),
          "batch descriptors");
  if (p->gexec) {
    (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
  }
  return SL_OK;
}

// Options of a batched run for `dim`-dimensional placements: a fixed factor,
// the Jacobi step, no traces.
sl_status batch_options(int dim, const sl_options* o, BatchParams* bp) {
  sl_status s = check_options(o);
  if (s != SL_OK) return s;
  if (o->dim != dim) return fail(SL_EINVAL, "options dim %d differs from the plan's %d", o->dim, dim);
  if (o->trace || o->xtrace) return fail(SL_EINVAL, "traces are not available for batched layouts");
  if (o->strategy != SL_OMEGA_FIXED || o->omega_vertex)
    return fail(SL_EINVAL, "batched layouts take a fixed relaxation factor");
  if (o->ordering != SL_ORDER_JACOBI) return fail(SL_ENOTSUP, "batched layouts use the Jacobi step");
  bp->omega_p = o->omega - 1.0;
  bp->tol = o->tol;
  bp->max_iter = o->max_iter;
  bp->safeguard = o->safeguard;
  return SL_OK;
}

sl_status batch_params(const sl_batch_plan* p, const sl_options* o, BatchParams* bp) {
  return batch_options(p->dim, o, bp);
}

// Time one launch over the graphs listed in `order` (device), in ms.
sl_status batch_time(sl_batch_plan* p, float* X, const int32_t* order, int count, const BatchParams& bp, float* ms) {
  HIP_TRY(launch_batch_reset(p->queue, p->ps), "reset kernel");
  HIP_TRY(hipEventRecord(p->ev_a, p->ps), "hipEventRecord");
  HIP_TRY(launch_batch_layout(p->dim, p->threads, batch_blocks(p, count), p->graphs, order, count, p->queue, p->d,
                              p->W, X, p->res, bp, p->ps),
          "batch layout kernel");
  HIP_TRY(hipEventRecord(p->ev_b, p->ps), "hipEventRecord");
  HIP_TRY(hipEventSynchronize(p->ev_b), "hipEventSynchronize");
  HIP_TRY(hipEventElapsedTime(ms, p->ev_a, p->ev_b), "hipEventElapsedTime");
  return SL_OK;
}

}  // namespace

extern "C" {

sl_status sl_batch_plan_create(const sl_batch* b, int32_t dim, void* stream, sl_batch_plan** out) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    if (!out) return fail(SL_EINVAL, "out is NULL");
    *out = nullptr;
    sl_status s = check_batch(b);
    if (s != SL_OK) return s;
    if (dim != 2 && dim != 3) return fail(SL_EINVAL, "dim = %d, expected 2 or 3", dim);
    sl_batch_plan* p = new (std::nothrow) sl_batch_plan();
    if (!p) return fail(SL_ENOMEM, "host allocation failed");
    auto bail = [&](sl_status st) {
      free_batch(p);
      delete p;
      return st;
    };
    p->ngraphs = b->num_graphs;
    p->dim = dim;
    p->n_total = b->num_graphs > 0 ? b->graph_ptr[b->num_graphs] : 0;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->ps, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&p->ev_a);
    if (e == hipSuccess) e = hipEventCreate(&p->ev_b);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_sync, hipEventDisableTiming);
    if (e != hipSuccess) return bail(hip_fail(e, "batch plan setup"));
    int64_t d_bytes = 0, w_total = 0;
    p->hgraphs.resize(p->ngraphs);
    for (int g = 0; g < p->ngraphs; ++g) {
      BatchGraph& G = p->hgraphs[g];
      G.n = (int32_t)(b->graph_ptr[g + 1] - b->graph_ptr[g]);
      G.n_pad = std::max(kRowBlock, round_up(G.n, kRowBlock));
      G.slices = default_slices(G.n_pad, p->threads);
      G.pad = 0;
      G.d_off = d_bytes;
      G.v_off = b->graph_ptr[g];
      G.w_off = w_total;
      d_bytes += (int64_t)G.n_pad * G.n_pad;
      w_total += G.n_pad;
    }
    p->horder.resize(p->ngraphs);
    for (int g = 0; g < p->ngraphs; ++g) p->horder[g] = g;
    std::stable_sort(p->horder.begin(), p->horder.end(),
                     [&](int a, int c) { return p->hgraphs[a].n_pad > p->hgraphs[c].n_pad; });
    p->hres.resize(p->ngraphs);
    const size_t ng1 = std::max(1, p->ngraphs);
    e = hipMalloc(&p->graphs, sizeof(BatchGraph) * ng1);
    if (e == hipSuccess) e = hipMalloc(&p->order, sizeof(int32_t) * ng1);
    if (e == hipSuccess) e = hipMalloc(&p->queue, sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&p->status, sizeof(int32_t) * ng1);
    if (e == hipSuccess) e = hipMalloc(&p->d, std::max<int64_t>(d_bytes, 1));
    if (e == hipSuccess) e = hipMalloc(&p->W, sizeof(double) * std::max<int64_t>(w_total, 1));
    if (e == hipSuccess) e = hipMalloc(&p->res, sizeof(BatchResult) * ng1);
    if (e != hipSuccess) return bail(hip_fail(e, "batch plan allocation"));
    if (p->ngraphs == 0) {
      *out = p;
      return SL_OK;
    }
    int64_t* rp = nullptr;
    int32_t* ci = nullptr;
    e = hipMalloc(&rp, sizeof(int64_t) * (p->n_total + 1));
    if (e == hipSuccess) e = hipMalloc(&ci, sizeof(int32_t) * std::max<int64_t>(b->nnz, 1));
    if (e == hipSuccess) e = hipEventRecord(p->ev_sync, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->ps, p->ev_sync, 0);
    if (e == hipSuccess) e = hipEventRecord(p->ev_a, p->ps);
    if (e == hipSuccess) e = hipMemsetAsync(p->d, 0, d_bytes, p->ps);
    if (e == hipSuccess) e = hipMemsetAsync(p->status, 0, sizeof(int32_t) * p->ngraphs, p->ps);
    if (e == hipSuccess)
      e = hipMemcpyAsync(rp, b->row_ptr, sizeof(int64_t) * (p->n_total + 1), hipMemcpyHostToDevice, p->ps);
    if (e == hipSuccess && b->nnz > 0)
      e = hipMemcpyAsync(ci, b->col_idx, sizeof(int32_t) * b->nnz, hipMemcpyHostToDevice, p->ps);
    if (e == hipSuccess)
      e = hipMemcpyAsync(p->order, p->horder.data(), sizeof(int32_t) * p->ngraphs, hipMemcpyHostToDevice, p->ps);
    if (e == hipSuccess)
      e = hipMemcpyAsync(p->graphs, p->hgraphs.data(), sizeof(BatchGraph) * p->ngraphs, hipMemcpyHostToDevice, p->ps);
    if (e == hipSuccess) e = launch_batch_reset(p->queue, p->ps);
    if (e == hipSuccess)
      e = launch_batch_distances(512, std::max(1, std::min(p->ngraphs, p->cus)), p->graphs, p->order, p->ngraphs,
                                 p->queue, rp, ci, p->d, p->W, p->status, p->ps);
    if (e == hipSuccess) e = hipEventRecord(p->ev_b, p->ps);
    std::vector<int32_t> hstatus(p->ngraphs, 0);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hstatus.data(), p->status, sizeof(int32_t) * p->ngraphs, hipMemcpyDeviceToHost, p->ps);
    if (e == hipSuccess) e = hipStreamSynchronize(p->ps);
    (void)hipFree(rp);
    (void)hipFree(ci);
    if (e != hipSuccess) return bail(hip_fail(e, "batch distances"));
    for (int g = 0; g < p->ngraphs; ++g)
      if (hstatus[g] != 0) return bail(fail(SL_ERANGE, "graph %d has a distance above 255 hops", g));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p->ev_a, p->ev_b);
    p->plan_ms = ms;
    *out = p;
    return SL_OK;
  });
}

sl_status sl_batch_plan_destroy(sl_batch_plan* p) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    if (!p) return SL_OK;
    (void)hipStreamSynchronize(p->ps);
    free_batch(p);
    delete p;
    return SL_OK;
  });
}

sl_status sl_batch_plan_tune(sl_batch_plan* p, const float* X, const sl_options* o, void* stream, int32_t* config) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    if (!p) return fail(SL_EINVAL, "plan is NULL");
    BatchParams bp{};
    sl_status s = batch_params(p, o, &bp);
    if (s != SL_OK) return s;
    if (p->ngraphs == 0 || p->n_total == 0) return SL_OK;
    if (!X) return fail(SL_EINVAL, "X is NULL");
    // The workgroup size is timed on whole runs to the caller's tolerance: a
    // launch lasts as long as its slowest graph, which short runs do not see
    // (a graph that needs many iterations runs faster on a larger workgroup
    // alone on its CU).  The slices per size class are timed on short runs.
    const BatchParams bp_run = bp;
    const bool whole = o->tol > 0.0;
    bp.tol = 0.0;
    bp.max_iter = std::max(1, std::min(o->max_iter, 8));
    const size_t xbytes = sizeof(float) * (size_t)p->n_total * p->dim;
    float* tmp = nullptr;
    int32_t* sub = nullptr;
    HIP_TRY(hipMalloc(&tmp, xbytes), "tuning buffer");
    if (hipMalloc(&sub, sizeof(int32_t) * p->ngraphs) != hipSuccess) {
      (void)hipFree(tmp);
      return fail(SL_ENOMEM, "tuning buffer");
    }
    auto cleanup = [&]() {
      (void)hipStreamSynchronize(p->ps);
      (void)hipFree(tmp);
      (void)hipFree(sub);
    };
    auto timed = [&](const int32_t* order, int count, const BatchParams& params, float* ms) -> sl_status {
      HIP_TRY(hipMemcpyAsync(tmp, X, xbytes, hipMemcpyDeviceToDevice, p->ps), "tuning copy");
      return batch_time(p, tmp, order, count, params, ms);
    };
    if ((s = join_from_stream(p->ps, p->ev_sync, (hipStream_t)stream)) != SL_OK) {
      cleanup();
      return s;
    }
    // 1. workgroup size, with the default slices for each
    int best_t = p->threads;
    float best_ms = 1e30f;
    for (int t : {256, 512, 1024}) {
      p->threads = t;
      for (auto& G : p->hgraphs) G.slices = default_slices(G.n_pad, t);
      if ((s = batch_upload_graphs(p)) != SL_OK) break;
      float ms = 0.f;
      if ((s = timed(p->order, p->ngraphs, whole ? bp_run : bp, &ms)) != SL_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        best_t = t;
      }
    }
    if (s != SL_OK) {
      cleanup();
      return s;
    }
    p->threads = best_t;
    for (auto& G : p->hgraphs) G.slices = default_slices(G.n_pad, best_t);
    // 2. column slices per size class, timed on that class alone
    int chosen[kBatchClasses] = {0};
    for (int c = 0; c < kBatchClasses && s == SL_OK; ++c) {
      const int n_pad = (c + 1) * kRowBlock;
      std::vector<int32_t> members;
      for (int g : p->horder)
        if (p->hgraphs[g].n_pad == n_pad) members.push_back(g);
      if (members.empty()) continue;
      if ((s = hip_try_copy(sub, members.data(), sizeof(int32_t) * members.size(), p->ps)) != SL_OK) break;
      int best_s = default_slices(n_pad, best_t);
      float best = 1e30f;
      for (int cand : {1, 2, 4, 8, 16}) {
        if (!slices_ok(n_pad, cand)) continue;
        for (int g : members) p->hgraphs[g].slices = cand;
        if ((s = batch_upload_graphs(p)) != SL_OK) break;
        float ms = 0.f;
        if ((s = timed(sub, (int)members.size(), bp, &ms)) != SL_OK) break;
        if (ms < best) {
          best = ms;
          best_s = cand;
        }
      }
      for (int g : members) p->hgraphs[g].slices = best_s;
      chosen[c] = best_s;
    }
    if (s == SL_OK) s = batch_upload_graphs(p);
    cleanup();
    if (s != SL_OK) return s;
    if (config) {
      config[0] = p->threads;
      for (int c = 0; c < kBatchClasses; ++c) config[1 + c] = chosen[c];
    }
    return join_to_stream(p->ps, p->ev_sync, (hipStream_t)stream);
  });
}

sl_status sl_batch_plan_run(sl_batch_plan* p, float* X, const sl_options* o, void* stream, sl_result* per_graph,
                            sl_result* total) {
  return guarded([&]() -> sl_status {
    g_err.clear();
    if (!p) return fail(SL_EINVAL, "plan is NULL");
    BatchParams bp{};
    sl_status s = batch_params(p, o, &bp);
    if (s != SL_OK) return s;
    sl_result tot{};
    tot.plan_ms = p->plan_ms;
    tot.converged = 1;
    if (p->ngraphs > 0 && p->n_total == 0)  // graphs without vertices: converged, no iterations
      for (BatchResult& r : p->hres) r = BatchResult{0, 1, 0, 0, 0.0, 0.0};
    if (p->ngraphs > 0 && p->n_total > 0) {
      if (!X) return fail(SL_EINVAL, "X is NULL");
      if ((s = join_from_stream(p->ps, p->ev_sync, (hipStream_t)stream)) != SL_OK) return s;
      std::vector<double> key = {(double)p->threads, bp.omega_p, bp.tol, (double)bp.max_iter, (double)bp.safeguard,
                                 (double)(uintptr_t)X};
      if (!p->gexec || key != p->gkey) {
        if (p->gexec) {
          (void)hipGraphExecDestroy(p->gexec);
          p->gexec = nullptr;
        }
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(p->ps, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        hipError_t le = launch_batch_reset(p->queue, p->ps);
        if (le == hipSuccess)
          le = launch_batch_layout(p->dim, p->threads, batch_blocks(p, p->ngraphs), p->graphs, p->order, p->ngraphs,
                                   p->queue, p->d, p->W, X, p->res, bp, p->ps);
        hipError_t ce = hipStreamEndCapture(p->ps, &graph);
        if (le != hipSuccess || ce != hipSuccess) {
          if (graph) (void)hipGraphDestroy(graph);
          return hip_fail(le != hipSuccess ? le : ce, "batch graph capture");
        }
        hipError_t ie = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
          p->gexec = nullptr;
          return hip_fail(ie, "hipGraphInstantiate");
        }
        p->gkey = key;
      }
      HIP_TRY(hipEventRecord(p->ev_a, p->ps), "hipEventRecord");
      HIP_TRY(hipGraphLaunch(p->gexec, p->ps), "hipGraphLaunch");
      HIP_TRY(hipEventRecord(p->ev_b, p->ps), "hipEventRecord");
      HIP_TRY(hipMemcpyAsync(p->hres.data(), p->res, sizeof(BatchResult) * p->ngraphs, hipMemcpyDeviceToHost, p->ps),
              "batch results");
      HIP_TRY(hipStreamSynchronize(p->ps), "hipStreamSynchronize");
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, p->ev_a, p->ev_b);
      tot.run_ms = ms;
      if ((s = join_to_stream(p->ps, p->ev_sync, (hipStream_t)stream)) != SL_OK) return s;
    }
    int bad = -1;
    for (int g = 0; g < p->ngraphs; ++g) {
      const BatchResult& r = p->hres[g];
      if (per_graph) {
        sl_result& o2 = per_graph[g];
        o2 = sl_result{};
        o2.iterations = r.iterations;
        o2.converged = r.converged;
        o2.rejected = r.rejected;
        o2.residual = r.residual;
        o2.stress = r.stress;
        o2.plan_ms = p->plan_ms;
        o2.run_ms = tot.run_ms;
        o2.rel_stress_drop = std::nan("");
      }
      tot.iterations = std::max(tot.iterations, r.iterations);
      tot.converged = tot.converged && r.converged;
      tot.rejected += r.rejected;
      tot.residual = std::max(tot.residual, r.residual);
      if (r.status != 0 && bad < 0) bad = g;
    }
    tot.rel_stress_drop = std::nan("");
    if (total) *total = tot;
    if (bad >= 0) return fail(SL_ENUMERIC, "graph %d: non-finite coordinate; its X holds the last finite iterate", bad);
    return SL_OK;
  });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Helpers for entry points defined in other files of the library: the same
// thread-local error text (sl_last_error) and option checks.
// ---------------------------------------------------------------------------
namespace sl {

void api_clear_error() { g_err.clear(); }
sl_status api_error(sl_status st, const char* msg) { return fail(st, "%s", msg); }
sl_status api_hip_error(hipError_t e, const char* what) { return hip_fail(e, what); }
sl_status api_batch_options(int dim, const sl_options* o, BatchParams* bp) { return batch_options(dim, o, bp); }

}  // namespace sl
