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
#include <string>
#include <vector>

using namespace sl;

namespace {

thread_local std::string g_err;

sl_status fail(sl_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

sl_status hip_fail(hipError_t e, const char* what) {
  const sl_status st = (e == hipErrorOutOfMemory) ? SL_ENOMEM : SL_EDEVICE;
  return fail(st, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                       \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// ---------------------------------------------------------------------------
// Host-side validation (no HIP calls)
// ---------------------------------------------------------------------------
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
  if (g->edge_len) {
    for (int64_t e = 0; e < g->nnz; ++e)
      if (!(std::isfinite(g->edge_len[e]) && g->edge_len[e] > 0.f))
        return fail(SL_EINVAL, "edge_len[%lld] is not a positive finite number", (long long)e);
    return fail(SL_ENOTSUP, "edge lengths (weighted distances) are not supported by this build");
  }
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
  if (o->flags & ~(SL_FLAG_TRACE_STRESS | SL_FLAG_NO_GRAPH)) return fail(SL_EINVAL, "unknown flag bits");
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
  uint8_t* d = nullptr;         // n_pad^2 bytes, tile-major
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
  int nsg = 0;
  DevState* st = nullptr;       // loop state
  DevState* st_eval = nullptr;  // state for stand-alone stress passes
  DevState* host_st = nullptr;  // pinned mirror
  double plan_ms = 0.0;
  // captured chunk of iterations, rebuilt when the loop parameters change
  hipGraphExec_t gexec = nullptr;
  std::vector<double> gkey;
};

namespace {

sl_status free_plan_memory(sl_plan* p) {
  (void)hipFree(p->d);
  (void)hipFree(p->W);
  (void)hipFree(p->Xb);
  (void)hipFree(p->Eb);
  (void)hipFree(p->items);
  (void)hipFree(p->fpart);
  (void)hipFree(p->spart);
  (void)hipFree(p->red);
  (void)hipFree(p->sgpart);
  (void)hipFree(p->st);
  (void)hipFree(p->st_eval);
  if (p->host_st) (void)hipHostFree(p->host_st);
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->ev_a) (void)hipEventDestroy(p->ev_a);
  if (p->ev_b) (void)hipEventDestroy(p->ev_b);
  if (p->ev_sync) (void)hipEventDestroy(p->ev_sync);
  if (p->ps) (void)hipStreamDestroy(p->ps);
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

// Multi-source BFS, bfs_sources_per_sweep() sources per sweep, then W.
// Distances above 255 hops are refused (SL_ERANGE).
sl_status build_distances(sl_plan* p, const sl_graph* g) {
  const int n = p->n;
  HIP_TRY(hipMemsetAsync(p->d, 0, (size_t)p->n_pad * p->n_pad, p->ps), "hipMemsetAsync(d)");
  if (n > 1 && g->nnz > 0) {
    // source row of every CSR entry, for the edge-parallel gather
    std::vector<int32_t> erow((size_t)g->nnz);
    for (int v = 0; v < n; ++v)
      for (int64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) erow[(size_t)e] = v;
    int32_t *er = nullptr, *ci = nullptr;
    uint64_t *fr = nullptr, *vis = nullptr, *nx = nullptr, *acc = nullptr;
    int32_t* flag = nullptr;
    int32_t* hflag = nullptr;
    sl_status status = SL_OK;
    auto cleanup = [&]() {
      (void)hipStreamSynchronize(p->ps);
      (void)hipFree(er);
      (void)hipFree(ci);
      (void)hipFree(fr);
      (void)hipFree(vis);
      (void)hipFree(nx);
      (void)hipFree(acc);
      (void)hipFree(flag);
      if (hflag) (void)hipHostFree(hflag);
    };
    hipError_t e = hipSuccess;
    const size_t words = (size_t)n * bfs_words();
    if (e == hipSuccess) e = hipMalloc(&er, sizeof(int32_t) * g->nnz);
    if (e == hipSuccess) e = hipMalloc(&ci, sizeof(int32_t) * g->nnz);
    if (e == hipSuccess) e = hipMalloc(&fr, sizeof(uint64_t) * words);
    if (e == hipSuccess) e = hipMalloc(&vis, sizeof(uint64_t) * words);
    if (e == hipSuccess) e = hipMalloc(&nx, sizeof(uint64_t) * words);
    if (e == hipSuccess) e = hipMalloc(&acc, sizeof(uint64_t) * words);
    if (e == hipSuccess) e = hipMalloc(&flag, sizeof(int32_t));
    if (e == hipSuccess) e = hipHostMalloc(&hflag, sizeof(int32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemcpyAsync(er, erow.data(), sizeof(int32_t) * g->nnz, hipMemcpyHostToDevice, p->ps);
    if (e == hipSuccess) e = hipMemcpyAsync(ci, g->col_idx, sizeof(int32_t) * g->nnz, hipMemcpyHostToDevice, p->ps);
    if (e != hipSuccess) {
      cleanup();
      return hip_fail(e, "distance buffers");
    }
    const int sweep = bfs_sources_per_sweep();
    for (int base = 0; base < n && status == SL_OK && e == hipSuccess; base += sweep) {
      e = launch_bfs_init(fr, vis, acc, n, base, p->ps);
      for (int level = 1; e == hipSuccess; ++level) {
        const int write = level <= 255;
        e = hipMemsetAsync(flag, 0, sizeof(int32_t), p->ps);
        if (e == hipSuccess)
          e = launch_bfs_level(er, ci, g->nnz, fr, acc, vis, nx, p->d, n, p->sp.ng, base, level, write, flag, p->ps);
        if (e == hipSuccess) e = hipMemcpyAsync(hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, p->ps);
        if (e == hipSuccess) e = hipStreamSynchronize(p->ps);
        if (e != hipSuccess || *hflag == 0) break;
        if (!write) {
          status = fail(SL_ERANGE, "a graph distance exceeds 255 hops (sources %d..%d)", base, base + sweep - 1);
          break;
        }
        std::swap(fr, nx);
      }
    }
    cleanup();
    if (e != hipSuccess) return hip_fail(e, "breadth-first search");
    if (status != SL_OK) return status;
  }
  HIP_TRY(launch_weights(p->d, p->W, p->sp, n, p->ps), "weights kernel");
  return SL_OK;
}

sl_status enqueue_iteration(sl_plan* p, const LoopParams& lp, const sl_options* o) {
  HIP_TRY(launch_force(p->dim, lp.stress != 0, p->d, p->Xb, p->stride, p->st, p->fpart, p->spart, p->sp, p->n_pad,
                       p->ps),
          "force kernel");
  HIP_TRY(launch_update(p->dim, lp, p->fpart, p->spart, p->W, p->Xb, p->stride, p->Eb, p->st, p->red, p->ps),
          "update kernel");
  if (lp.safeguard && lp.omega_p != 0.0)
    HIP_TRY(launch_sgdelta(p->dim, p->d, p->Xb, p->stride, p->Eb, p->items, p->nsg, p->st, p->sgpart, p->sp,
                           p->ps),
            "safeguard kernel");
  HIP_TRY(launch_select(p->dim, lp, p->red, p->nred, p->sgpart, p->nsg, p->st, o->trace, p->ps), "select kernel");
  if (o->xtrace) HIP_TRY(launch_record(p->Xb, p->stride, p->st, o->xtrace, p->n, p->dim, p->ps), "record kernel");
  return SL_OK;
}

sl_status stress_pass(sl_plan* p, int cur, double* f) {
  DevState* h = p->host_st;
  std::memset(h, 0, sizeof(DevState));
  h->cur = cur;
  HIP_TRY(hipMemcpyAsync(p->st_eval, h, sizeof(DevState), hipMemcpyHostToDevice, p->ps), "state upload");
  HIP_TRY(launch_force(p->dim, true, p->d, p->Xb, p->stride, p->st_eval, p->fpart, p->spart, p->sp, p->n_pad,
                       p->ps),
          "force kernel");
  HIP_TRY(launch_stress_sum(p->spart, p->sp.slices, p->n_pad, p->st_eval, p->ps), "stress kernel");
  HIP_TRY(hipMemcpyAsync(h, p->st_eval, sizeof(DevState), hipMemcpyDeviceToHost, p->ps), "state download");
  HIP_TRY(hipStreamSynchronize(p->ps), "hipStreamSynchronize");
  *f = h->stress;
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
  g_err.clear();
  sl_status s = check_graph(g);
  if (s != SL_OK) return s;
  if (opt) return check_options(opt);
  return SL_OK;
}

sl_status sl_plan_create(const sl_graph* g, int32_t dim, void* stream, sl_plan** out) {
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
  if (e == hipSuccess) e = hipMalloc(&p->d, (size_t)p->n_pad * p->n_pad);
  if (e == hipSuccess) e = hipMalloc(&p->W, sizeof(double) * p->n_pad);
  if (e == hipSuccess) e = hipMalloc(&p->Xb, sizeof(float) * 3 * p->stride);
  if (e == hipSuccess) e = hipMalloc(&p->Eb, sizeof(float) * p->stride);
  if (e == hipSuccess) e = hipMalloc(&p->items, sizeof(int4) * items.size());
  if (e == hipSuccess) e = hipMalloc(&p->fpart, sizeof(double) * p->sp.slices * 3 * p->n_pad);
  if (e == hipSuccess) e = hipMalloc(&p->spart, sizeof(double) * p->sp.slices * p->n_pad);
  if (e == hipSuccess) e = hipMalloc(&p->red, sizeof(double) * 8 * p->nred);
  if (e == hipSuccess) e = hipMalloc(&p->sgpart, sizeof(double) * p->nsg);
  if (e == hipSuccess) e = hipMalloc(&p->st, sizeof(DevState));
  if (e == hipSuccess) e = hipMalloc(&p->st_eval, sizeof(DevState));
  if (e == hipSuccess) e = hipHostMalloc(&p->host_st, sizeof(DevState), hipHostMallocDefault);
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
}

sl_status sl_plan_destroy(sl_plan* p) {
  g_err.clear();
  if (!p) return SL_OK;
  (void)hipStreamSynchronize(p->ps);
  free_plan_memory(p);
  delete p;
  return SL_OK;
}

sl_status sl_plan_run(sl_plan* p, float* X, const sl_options* o, void* stream, sl_result* out) {
  g_err.clear();
  if (!p) return fail(SL_EINVAL, "plan is NULL");
  sl_status s = check_options(o);
  if (s != SL_OK) return s;
  if (o->dim != p->dim) return fail(SL_EINVAL, "options dim %d differs from the plan's %d", o->dim, p->dim);
  if (!X && p->n > 0) return fail(SL_EINVAL, "X is NULL");
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

  if ((s = join_from(p, user)) != SL_OK) return s;
  if (p->n > 0) HIP_TRY(launch_pack_in(X, p->Xb, p->n, p->n_pad, p->dim, p->ps), "pack kernel");
  DevState* h = p->host_st;
  std::memset(h, 0, sizeof(DevState));
  h->max_iter = o->max_iter;
  h->done = (o->max_iter == 0 || p->n <= 1) ? 1 : 0;
  h->converged = p->n <= 1 ? 1 : 0;
  HIP_TRY(hipMemcpyAsync(p->st, h, sizeof(DevState), hipMemcpyHostToDevice, p->ps), "state upload");

  int chunk = o->check_every > 0 ? o->check_every : (p->n <= 8192 ? 32 : 4);
  chunk = std::max(1, std::min(chunk, std::max(1, o->max_iter)));
  const bool use_graph = !(o->flags & SL_FLAG_NO_GRAPH);
  if (use_graph) {
    std::vector<double> key = {(double)p->dim, lp.omega_p, lp.tol, (double)lp.safeguard, (double)lp.stress,
                               (double)chunk, (double)(uintptr_t)o->trace, (double)(uintptr_t)o->xtrace};
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
  const int max_launches = o->max_iter / chunk + 2;
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
  double f = 0.0;
  if (p->n > 1 && (s = stress_pass(p, fin.cur, &f)) != SL_OK) return s;
  res.stress = f;
  if ((s = join_to(p, user)) != SL_OK) return s;
  if (out) *out = res;
  if (fin.status != 0)
    return fail(SL_ENUMERIC, "non-finite coordinate at iteration %d; X holds the last finite iterate", fin.iter + 1);
  return SL_OK;
}

sl_status sl_plan_stress(sl_plan* p, const float* X, int32_t dim, void* stream, double* f) {
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
}

sl_status sl_plan_profile(sl_plan* p, const float* X, int32_t dim, double omega, int32_t reps, void* stream,
                          double* ms) {
  g_err.clear();
  if (!p || !ms) return fail(SL_EINVAL, "plan or ms is NULL");
  if (dim != p->dim) return fail(SL_EINVAL, "dim %d differs from the plan's %d", dim, p->dim);
  if (!X && p->n > 0) return fail(SL_EINVAL, "X is NULL");
  if (reps < 1) return fail(SL_EINVAL, "reps must be >= 1");
  if (!(std::isfinite(omega) && omega > 0.0 && omega <= 16.0)) return fail(SL_EINVAL, "omega outside (0, 16]");
  sl_status s = join_from(p, (hipStream_t)stream);
  if (s != SL_OK) return s;
  for (int k = 0; k < 4; ++k) ms[k] = 0.0;
  if (p->n <= 1) return SL_OK;
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
  HIP_TRY(launch_pack_in(X, p->Xb, p->n, p->n_pad, p->dim, p->ps), "pack kernel");
  DevState* h = p->host_st;
  std::memset(h, 0, sizeof(DevState));
  h->max_iter = INT32_MAX;
  HIP_TRY(hipMemcpyAsync(p->st, h, sizeof(DevState), hipMemcpyHostToDevice, p->ps), "state upload");
  for (int which = 0; which < 4; ++which) {
    for (int r = -1; r < reps; ++r) {  // one untimed launch first
      if (r == 0) HIP_TRY(hipEventRecord(p->ev_a, p->ps), "hipEventRecord");
      switch (which) {
        case 0:
          HIP_TRY(launch_force(p->dim, false, p->d, p->Xb, p->stride, p->st, p->fpart, p->spart, p->sp, p->n_pad,
                               p->ps), "force kernel");
          break;
        case 1:
          HIP_TRY(launch_update(p->dim, lp, p->fpart, p->spart, p->W, p->Xb, p->stride, p->Eb, p->st, p->red,
                                p->ps),
                  "update kernel");
          break;
        case 2:
          HIP_TRY(launch_sgdelta(p->dim, p->d, p->Xb, p->stride, p->Eb, p->items, p->nsg, p->st, p->sgpart,
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
}

sl_status sl_plan_distance_rows(sl_plan* p, const int32_t* rows, int32_t nrows, void* stream, uint8_t* out) {
  g_err.clear();
  if (!p) return fail(SL_EINVAL, "plan is NULL");
  if (nrows < 0) return fail(SL_EINVAL, "nrows is negative");
  if (nrows == 0) return SL_OK;
  if (!rows || !out) return fail(SL_EINVAL, "rows or out is NULL");
  for (int k = 0; k < nrows; ++k)
    if (rows[k] < 0 || rows[k] >= p->n) return fail(SL_EINVAL, "row %d outside [0, n)", rows[k]);
  if (p->n == 0) return SL_OK;
  sl_status s = join_from(p, (hipStream_t)stream);
  if (s != SL_OK) return s;
  int32_t* drows = nullptr;
  uint8_t* dout = nullptr;
  const size_t bytes = (size_t)nrows * p->n;
  hipError_t e = hipMalloc(&drows, sizeof(int32_t) * nrows);
  if (e == hipSuccess) e = hipMalloc(&dout, bytes);
  if (e == hipSuccess) e = hipMemcpyAsync(drows, rows, sizeof(int32_t) * nrows, hipMemcpyHostToDevice, p->ps);
  if (e == hipSuccess) e = launch_gather_rows(p->d, drows, nrows, p->n, p->sp.ng, dout, p->ps);
  if (e == hipSuccess) e = hipMemcpyAsync(out, dout, bytes, hipMemcpyDeviceToHost, p->ps);
  if (e == hipSuccess) e = hipStreamSynchronize(p->ps);
  (void)hipFree(drows);
  (void)hipFree(dout);
  if (e != hipSuccess) return hip_fail(e, "distance rows");
  return SL_OK;
}

sl_status sl_plan_weights(sl_plan* p, void* stream, double* W) {
  g_err.clear();
  if (!p || !W) return fail(SL_EINVAL, "plan or W is NULL");
  if (p->n == 0) return SL_OK;
  sl_status s = join_from(p, (hipStream_t)stream);
  if (s != SL_OK) return s;
  HIP_TRY(hipMemcpyAsync(W, p->W, sizeof(double) * p->n, hipMemcpyDeviceToHost, p->ps), "weights copy");
  HIP_TRY(hipStreamSynchronize(p->ps), "hipStreamSynchronize");
  return SL_OK;
}

sl_status sl_layout(const sl_graph* g, float* X, const sl_options* o, void* stream, sl_result* out) {
  g_err.clear();
  sl_status s = check_options(o);
  if (s != SL_OK) return s;
  sl_plan* p = nullptr;
  if ((s = sl_plan_create(g, o->dim, stream, &p)) != SL_OK) return s;
  s = sl_plan_run(p, X, o, stream, out);
  const std::string keep = g_err;
  sl_plan_destroy(p);
  g_err = keep;
  return s;
}

}  // extern "C"
