// Allocation-free batched layout (sl_batch_layout_noalloc): the batched path
// of sl_batch_plan_create + sl_batch_plan_run (same kernels, same launch
// shapes, untuned defaults) with every device buffer carved out of one static
// per-device array instead of hipMalloc, and every host buffer static.
//
// Device memory: `scratch`, a file-scope __device__ array of
// SL_NOALLOC_SCRATCH_BYTES.  Each GPU the library runs on holds its own copy
// at its own address from module load until the process ends.  Host code
// never passes the array's name to a kernel or a copy (on the host it is only
// a stand-in for the symbol): the first call on a device looks the device
// address up with hipGetSymbolAddress and keeps it per device.
//
// Concurrency: every call shares the device's array, which keeps the last
// call's contents, so a process-wide lock is held for the whole call; calls
// from several host threads run one after another.
#include "sorlayout.h"
#include "sl_internal.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

namespace sl {
// defined in sl_api.hip: the C ABI's thread-local error text and option checks
void api_clear_error();
sl_status api_error(sl_status st, const char* msg);
sl_status api_hip_error(hipError_t e, const char* what);
sl_status api_batch_options(int dim, const sl_options* o, BatchParams* bp);
}  // namespace sl

using namespace sl;

namespace {

static __device__ __align__(256) unsigned char scratch[SL_NOALLOC_SCRATCH_BYTES];

constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;
// each graph needs at least one 64 x 64 block of distance bytes
constexpr int kMaxGraphs = (int)(SL_NOALLOC_SCRATCH_BYTES / ((size_t)kRowBlock * kRowBlock));
constexpr int kAdjWords = kBatchMaxN / 64;

std::mutex g_lock;                  // held for a whole call
unsigned char* g_dev_ptr[kMaxDevices] = {nullptr};  // device address of `scratch`, per device
int g_dev_cus[kMaxDevices] = {0};

// Host staging, static (used under g_lock only).
BatchGraph h_graphs[kMaxGraphs];
int32_t h_order[kMaxGraphs];
int32_t h_status[kMaxGraphs];
BatchResult h_res[kMaxGraphs];
uint64_t h_adj[kBatchMaxN * kAdjWords];  // one graph's adjacency bits, for validation

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// The entry point's body runs through this, so that no C++ exception (the
// lock's, say) crosses the C ABI.
template <class F>
sl_status guarded_call(F&& body) noexcept {
  try {
    return body();
  } catch (...) {
    return api_error(SL_EDEVICE, "host runtime error");
  }
}

sl_status errorf(sl_status st, const char* fmt, long long a, long long b = 0, long long c = 0) {
  char msg[256];
  snprintf(msg, sizeof msg, fmt, a, b, c);
  return api_error(st, msg);
}

// Edges of graph g (vertices v0 .. v0 + n - 1) through the adjacency bits of
// h_adj, which the caller clears afterwards.
sl_status check_graph_bits(const sl_batch* b, int g, int64_t v0, int64_t n) {
  for (int64_t v = 0; v < n; ++v) {
    uint64_t* row = h_adj + v * kAdjWords;
    for (int64_t e = b->row_ptr[v0 + v]; e < b->row_ptr[v0 + v + 1]; ++e) {
      const int64_t u = (int64_t)b->col_idx[e] - v0;
      if (u < 0 || u >= n) return errorf(SL_EINVAL, "edge (%lld, %lld) leaves graph %lld", v0 + v, b->col_idx[e], g);
      if (u == v) return errorf(SL_EINVAL, "self loop at vertex %lld", v0 + v);
      const uint64_t bit = 1ull << (u % 64);
      if (row[u / 64] & bit) return errorf(SL_EINVAL, "duplicate edge (%lld, %lld)", v0 + v, v0 + u);
      row[u / 64] |= bit;
    }
  }
  for (int64_t v = 0; v < n; ++v)
    for (int64_t e = b->row_ptr[v0 + v]; e < b->row_ptr[v0 + v + 1]; ++e) {
      const int64_t u = (int64_t)b->col_idx[e] - v0;
      if (!(h_adj[u * kAdjWords + v / 64] & (1ull << (v % 64))))
        return errorf(SL_EINVAL, "graph is not symmetric: (%lld, %lld) has no reverse entry", v0 + v, v0 + u);
    }
  return SL_OK;
}

// The checks of a batch that sl_batch_plan_create makes, without a heap
// allocation: CSR shape, ids inside their own graph, no self loops or
// duplicates, symmetry (an adjacency bitmap of one graph at a time).
sl_status check_batch_static(const sl_batch* b) {
  if (!b) return api_error(SL_EINVAL, "batch is NULL");
  if (b->num_graphs < 0) return api_error(SL_EINVAL, "num_graphs is negative");
  if (b->num_graphs > kMaxGraphs)
    return errorf(SL_EINVAL, "%lld graphs, more than the %lld the scratch array can hold", b->num_graphs, kMaxGraphs);
  if (b->num_graphs == 0) {
    if (b->nnz != 0) return api_error(SL_EINVAL, "empty batch with edges");
    return SL_OK;
  }
  if (!b->graph_ptr) return api_error(SL_EINVAL, "graph_ptr is NULL");
  if (b->graph_ptr[0] != 0) return api_error(SL_EINVAL, "graph_ptr[0] must be 0");
  for (int g = 0; g < b->num_graphs; ++g) {
    const int64_t n = b->graph_ptr[g + 1] - b->graph_ptr[g];
    if (n < 0) return errorf(SL_EINVAL, "graph_ptr decreases at graph %lld", g);
    if (n > SL_BATCH_MAX_N) return errorf(SL_EINVAL, "graph %lld has %lld vertices, more than %lld", g, n,
                                          SL_BATCH_MAX_N);
  }
  const int64_t n_total = b->graph_ptr[b->num_graphs];
  if (n_total > INT32_MAX) return api_error(SL_EINVAL, "too many vertices in the batch");
  if (n_total == 0) {
    if (b->nnz != 0) return api_error(SL_EINVAL, "empty batch with edges");
    return SL_OK;
  }
  if (!b->row_ptr) return api_error(SL_EINVAL, "row_ptr is NULL");
  if (b->nnz < 0) return api_error(SL_EINVAL, "nnz is negative");
  if (b->nnz > 0 && !b->col_idx) return api_error(SL_EINVAL, "col_idx is NULL");
  if (b->row_ptr[0] != 0) return errorf(SL_EINVAL, "row_ptr[0] = %lld, expected 0", b->row_ptr[0]);
  for (int64_t v = 0; v < n_total; ++v)
    if (b->row_ptr[v + 1] < b->row_ptr[v]) return errorf(SL_EINVAL, "row_ptr decreases at row %lld", v);
  if (b->row_ptr[n_total] != b->nnz)
    return errorf(SL_EINVAL, "row_ptr[n] = %lld differs from nnz = %lld", b->row_ptr[n_total], b->nnz);
  for (int g = 0; g < b->num_graphs; ++g) {
    const int64_t v0 = b->graph_ptr[g], n = b->graph_ptr[g + 1] - v0;
    const sl_status st = check_graph_bits(b, g, v0, n);
    std::memset(h_adj, 0, sizeof(uint64_t) * kAdjWords * (size_t)n);  // clean for the next graph and call
    if (st != SL_OK) return st;
  }
  return SL_OK;
}

// Device address of `scratch` and the CU count of the current device, found
// once per device (under g_lock).
sl_status device_scratch(unsigned char** ptr, int* cus) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return api_hip_error(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return errorf(SL_ENOTSUP, "device %lld beyond the %lld supported", dev, kMaxDevices);
  if (!g_dev_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return api_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
    int n = 0;
    e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return api_hip_error(e, "hipDeviceGetAttribute");
    g_dev_cus[dev] = n;
    g_dev_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *ptr = g_dev_ptr[dev];
  *cus = g_dev_cus[dev];
  return SL_OK;
}

}  // namespace

extern "C" {

sl_status sl_batch_layout_noalloc(const sl_batch* b, float* X, const sl_options* o, void* stream,
                                  sl_result* per_graph, sl_result* total) {
  return guarded_call([&]() -> sl_status {
    std::lock_guard<std::mutex> guard(g_lock);
    api_clear_error();
    sl_status s = check_batch_static(b);
    if (s != SL_OK) return s;
    if (!o) return api_error(SL_EINVAL, "options are NULL");
    BatchParams bp{};
    if ((s = api_batch_options(o->dim, o, &bp)) != SL_OK) return s;
    const int ng = b->num_graphs;
    const int dim = o->dim;
    const int64_t n_total = ng > 0 ? b->graph_ptr[ng] : 0;
    // descriptors as sl_batch_plan_create makes them: default slices of a
    // 512-thread workgroup, largest graph first
    constexpr int kThreads = 512;
    int64_t d_bytes = 0, w_total = 0;
    for (int g = 0; g < ng; ++g) {
      BatchGraph& G = h_graphs[g];
      G.n = (int32_t)(b->graph_ptr[g + 1] - b->graph_ptr[g]);
      G.n_pad = std::max(kRowBlock, (G.n + kRowBlock - 1) / kRowBlock * kRowBlock);
      G.slices = batch_default_slices(G.n_pad, kThreads);
      G.pad = 0;
      G.d_off = d_bytes;
      G.v_off = b->graph_ptr[g];
      G.w_off = w_total;
      d_bytes += (int64_t)G.n_pad * G.n_pad;
      w_total += G.n_pad;
      h_order[g] = g;
    }
    // largest n_pad first, ties in graph order (a stable order without a buffer)
    std::sort(h_order, h_order + ng, [](int a, int c) {
      return h_graphs[a].n_pad != h_graphs[c].n_pad ? h_graphs[a].n_pad > h_graphs[c].n_pad : a < c;
    });
    // carve the scratch array
    size_t off = 0;
    auto take = [&](size_t bytes) {
      const size_t at = off;
      off = align_up(off + std::max<size_t>(bytes, 1));
      return at;
    };
    const size_t o_graphs = take(sizeof(BatchGraph) * ng), o_order = take(sizeof(int32_t) * ng),
                 o_queue = take(sizeof(int32_t)), o_status = take(sizeof(int32_t) * ng),
                 o_res = take(sizeof(BatchResult) * ng), o_W = take(sizeof(double) * (size_t)w_total),
                 o_rp = take(sizeof(int64_t) * (size_t)(n_total + 1)), o_ci = take(sizeof(int32_t) * (size_t)b->nnz),
                 o_d = take((size_t)d_bytes);
    if (off > SL_NOALLOC_SCRATCH_BYTES)
      return errorf(SL_EINVAL, "the batch needs %lld bytes of device scratch, more than SL_NOALLOC_SCRATCH_BYTES = %lld",
                    (long long)off, (long long)SL_NOALLOC_SCRATCH_BYTES);
    sl_result tot{};
    tot.plan_ms = tot.run_ms = tot.rel_stress_drop = std::nan("");
    tot.converged = 1;
    if (ng > 0 && n_total > 0) {
      if (!X) return api_error(SL_EINVAL, "X is NULL");
      unsigned char* base = nullptr;
      int cus = 0;
      if ((s = device_scratch(&base, &cus)) != SL_OK) return s;
      const hipStream_t st = (hipStream_t)stream;
      BatchGraph* graphs = reinterpret_cast<BatchGraph*>(base + o_graphs);
      int32_t* order = reinterpret_cast<int32_t*>(base + o_order);
      int32_t* queue = reinterpret_cast<int32_t*>(base + o_queue);
      int32_t* status = reinterpret_cast<int32_t*>(base + o_status);
      BatchResult* res = reinterpret_cast<BatchResult*>(base + o_res);
      double* W = reinterpret_cast<double*>(base + o_W);
      int64_t* rp = reinterpret_cast<int64_t*>(base + o_rp);
      int32_t* ci = reinterpret_cast<int32_t*>(base + o_ci);
      uint8_t* d = base + o_d;
      // distances and weights (the plan's part), on the caller's stream
      hipError_t e = launch_fill_zero(d, (size_t)d_bytes, st);
      if (e == hipSuccess) e = launch_fill_zero(status, sizeof(int32_t) * ng, st);
      if (e == hipSuccess) e = hipMemcpyAsync(rp, b->row_ptr, sizeof(int64_t) * (n_total + 1), hipMemcpyHostToDevice, st);
      if (e == hipSuccess && b->nnz > 0)
        e = hipMemcpyAsync(ci, b->col_idx, sizeof(int32_t) * b->nnz, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(order, h_order, sizeof(int32_t) * ng, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(graphs, h_graphs, sizeof(BatchGraph) * ng, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = launch_batch_reset(queue, st);
      if (e == hipSuccess)
        e = launch_batch_distances(kThreads, std::max(1, std::min(ng, cus)), graphs, order, ng, queue, rp, ci, d, W,
                                   status, st);
      if (e == hipSuccess) e = hipMemcpyAsync(h_status, status, sizeof(int32_t) * ng, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return api_hip_error(e, "batch distances");
      for (int g = 0; g < ng; ++g)
        if (h_status[g] != 0) return errorf(SL_ERANGE, "graph %lld has a distance above 255 hops", g);
      // the layout (the run's part)
      e = launch_batch_reset(queue, st);
      if (e == hipSuccess)
        e = launch_batch_layout(dim, kThreads, batch_layout_blocks(dim, cus, ng), graphs, order, ng, queue, d, W, X, res,
                                bp, st);
      if (e == hipSuccess) e = hipMemcpyAsync(h_res, res, sizeof(BatchResult) * ng, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return api_hip_error(e, "batch layout");
    }
    int bad = -1;
    for (int g = 0; g < ng; ++g) {
      // graphs without vertices: converged, no iterations (as the kernel reports n <= 1)
      const BatchResult r = n_total > 0 ? h_res[g] : BatchResult{0, 1, 0, 0, 0.0, 0.0};
      if (per_graph) {
        sl_result& o2 = per_graph[g];
        o2 = sl_result{};
        o2.iterations = r.iterations;
        o2.converged = r.converged;
        o2.rejected = r.rejected;
        o2.residual = r.residual;
        o2.stress = r.stress;
        o2.plan_ms = o2.run_ms = o2.rel_stress_drop = std::nan("");
      }
      tot.iterations = std::max(tot.iterations, r.iterations);
      tot.converged = tot.converged && r.converged;
      tot.rejected += r.rejected;
      tot.residual = std::max(tot.residual, r.residual);
      if (r.status != 0 && bad < 0) bad = g;
    }
    if (total) *total = tot;
    if (bad >= 0)
      return errorf(SL_ENUMERIC, "graph %lld: non-finite coordinate; its X holds the last finite iterate", bad);
    return SL_OK;
  });
}

}  // extern "C"
