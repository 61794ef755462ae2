/*
 * sorlayout.h: C ABI of the MI355X (gfx950) library for SOR-accelerated
 * stress-majorization graph layout.
 *
 * Method: Wang & Wang, "A Fast Successive Over-Relaxation Algorithm for
 * Force-Directed Network Graph Drawing", Sci. China Inf. Sci. 55:677 (2012).
 *
 *   problem (Sec. 1, Sec. 2)  undirected G = (V, E), straight-line drawing,
 *                             placement X in R^{n x dim}
 *   stress (eq. 1)            f(X) = sum_{i<j} w_ij (||x_i - x_j|| - d_ij)^2,
 *                             d_ij = graph distance, w_ij = d_ij^-2 (Sec. 5.1)
 *   step H (Prop. 2.3, eq. 5) L^W X^H = L^X X, in one of two orderings:
 *                             SL_ORDER_JACOBI (default) applies one Jacobi
 *                             sweep of eq. 5 per iteration:
 *                             x_i^H = x_i + (1/W_i) sum_j w_ij (d_ij - r_ij) u_ij
 *                             SL_ORDER_EXACT solves eq. 5 (the paper's step,
 *                             Alg. 1/2, step H) by preconditioned conjugate
 *                             gradients
 *   SOR (Alg. 2, eq. 11)      X~ = X^H + (omega - 1)(X^H - X); keep X~ only if
 *                             f(X~) <= f(X^H) (Alg. 2, the safeguard)
 *   termination               res_k = ||X^H - X^k||_F / ||X^H - mean(X^H)||_F
 *                             <= tol (the paper leaves the test open: Alg. 1/2)
 *
 * omega is the classical relaxation factor: the paper's factor is omega - 1,
 * so omega = 1 is Algorithm 1 and the paper's 0.5, 1.0, 1.5 are omega = 1.5,
 * 2.0, 2.5.
 *
 * Conventions for every call
 *   - Every call returns sl_status (SL_OK = 0).  On failure sl_last_error()
 *     returns a message for the calling thread; it stays valid until the
 *     thread's next call into the library.
 *   - The caller owns every buffer it passes.  The library keeps no caller
 *     pointer after a call returns.  A plan owns its device memory (distances,
 *     weights, iterates, workspaces) until sl_plan_destroy.
 *   - Device work is queued on `stream` (a hipStream_t; NULL = the null
 *     stream) of the current HIP device.  Calls that return results to the
 *     host synchronize that stream before returning.
 *   - Validation errors (SL_EINVAL) are reported before any device work.
 */
#ifndef SORLAYOUT_H
#define SORLAYOUT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SL_OK = 0,
  SL_EINVAL = -1,    /* malformed graph or option                               */
  SL_ENOMEM = -2,    /* device or host allocation failed                       */
  SL_EDEVICE = -3,   /* a HIP call (or, rarely, the host runtime) failed       */
  SL_ERANGE = -4,    /* a finite graph distance exceeds 255 hops               */
  SL_ENUMERIC = -5,  /* a non-finite coordinate appeared during the iteration  */
  SL_ENOTSUP = -6    /* valid input the library does not handle               */
} sl_status;

/* Columns of one trace row (one row per iteration, doubles). */
#define SL_TRACE_COLS 7
/*   [0] res_k                      relative step ||X^H - X^k|| / ||X^H - mean||
 *   [1] accepted                   1 / 0 for the safeguard decision, -1 when no
 *                                  extrapolation is formed (omega == 1)
 *   [2] f(X~) - f(X^H)             summed pair by pair (0 when no safeguard is
 *                                  evaluated; NaN when the bounds [5], [6] decided)
 *   [3] paper's factor used        omega - 1 of this iteration (NaN with per-vertex
 *                                  factors)
 *   [4] f(X^k)                     stress at the iterate the step starts from
 *                                  (NaN unless SL_FLAG_TRACE_STRESS)
 *   [5] U >= f(X~) - f(X^H)        bounds formed by the force pass over unordered
 *   [6] L <= f(X~) - f(X^H)        pairs (SL_FLAG_SYM_FORCE with the fused
 *                                  safeguard): each pair's term w (r~ - r^H)
 *                                  (r~ + r^H - 2d) equals -c m - kappa delta^2 with
 *                                  c = 1/(d r~) - 1/d^2, m = r~^2 - r^H^2,
 *                                  kappa = 1/(d r~), delta = r~ - r^H, and
 *                                  delta^2 <= |e_i - e_j|^2 (e = X~ - X^H), so
 *                                  U = sum -c m and L = U - sum kappa |e_i - e_j|^2.
 *                                  U <= 0 keeps X~ and L > 0 keeps X^H without [2];
 *                                  otherwise [2] is summed and decides, and the
 *                                  next iterations sum [2] and U in the force
 *                                  pass itself ([6] NaN) until U <= 0 again.
 *                                  NaN when no bounds are formed                 */

/* Relaxation strategies (Sec. 5.2; per-vertex factors: Sec. 6, item 1).  Iterations
 * are numbered globally: iteration k of a call is iteration g = iter_offset + k. */
#define SL_OMEGA_FIXED 0     /* `omega` every iteration                                  */
#define SL_OMEGA_SCHEDULE 1  /* omega_schedule[g] at iteration g (a caller's sequence)   */
#define SL_OMEGA_ENUM 2      /* the paper's factor c = omega - 1 chosen each iteration as
                                the argmin of f(X^H + c (X^H - X^k)) over
                                c in {0, 0.5, ..., 9}; c = 0 keeps X^H (counted rejected) */
#define SL_OMEGA_AUTO 3      /* the probabilistic strategy (Sec. 5.2): the paper's factor of
                                iteration g is drawn by roulette from {0.5, 1.0, 1.5, 2.0}
                                with probabilities 0.3, 0.3, 0.2, 0.2, from the uniform
                                u = (z >> 11) 2^-53, z = output number g (from 0) of
                                SplitMix64 seeded with `seed` (Steele, Lea and Flood,
                                OOPSLA 2014): u < 0.3 -> 0.5, u < 0.6 -> 1.0,
                                u < 0.8 -> 1.5, else 2.0.  A run resumed with iter_offset
                                continues the sequence                                    */

/* Orderings of the step H (eq. 5). */
#define SL_ORDER_JACOBI 0    /* one Jacobi sweep: X^H = X^k + F / W                       */
#define SL_ORDER_EXACT 1     /* eq. 5 solved: conjugate gradients on L^W Y = L^X X^k from
                                Y = X^k, preconditioned by W, to ||r|| <= inner_tol ||r_0||;
                                L^W is singular, and the lowest-numbered vertex of each
                                connected component keeps its place (the paper fixes x_1,
                                Sec. 2: a translation of the same solution)               */

#define SL_FLAG_TRACE_STRESS 1u  /* evaluate f(X^k) every iteration into trace[4]  */
#define SL_FLAG_NO_GRAPH 2u      /* launch kernels one by one instead of replaying a
                                    captured HIP graph of `check_every` iterations */
#define SL_FLAG_SYM_FORCE 4u     /* evaluate the force pass once per unordered pair
                                    (F_j takes -c_ij (x_i - x_j), Newton's third law;
                                    the same sums in another order).  No stress trace
                                    (SL_ENOTSUP).  Hop-count and edge-length plans.
                                    The default, with the Jacobi step and no stress
                                    trace, from n_pad 24576 (16384 for a run that
                                    extrapolates with the safeguard, and for
                                    edge-length plans), in 2-D and 3-D: the faster
                                    pass there.  With SL_ORDER_EXACT it selects the
                                    L^W matvec of the conjugate gradients over
                                    unordered pairs (the default from n_pad 24576;
                                    the force pass there stays over ordered pairs).
                                    The first such run allocates the partial sums   */
#define SL_FLAG_ORDERED_FORCE 16u /* evaluate the force pass (and the exact step's
                                    L^W matvec) over every ordered pair from its row
                                    end (the default below those sizes, for the
                                    exact step's force pass and for stress traces).
                                    Not with SL_FLAG_SYM_FORCE (SL_EINVAL)           */
#define SL_FLAG_SEPARATE_SAFEGUARD 8u  /* evaluate f(X~) - f(X^H) in its own pass over
                                          unordered pairs and the next force pass
                                          after the decision.  Default (either
                                          ordering, a safeguard to evaluate, no
                                          enumeration or stress trace): the
                                          safeguard is summed inside the next
                                          iteration's force pass, taken at X~;
                                          when X~ is rejected the force pass at
                                          X^H runs again.  The same iterates. */
#define SL_FLAG_NO_FINAL_STRESS 32u  /* do not evaluate f of the returned placement
                                        (one pass over all pairs after the loop):
                                        sl_result.stress is NaN.  The iterates are
                                        the same.                                */

/* The graph G = (V, E) of the problem statement (Sec. 1), host memory, CSR.
 * Symmetric: (u, v) present iff (v, u) present.  Vertex ids 0 .. n-1.  No self
 * loops, no duplicate entries; neighbours of each row in any order. */
typedef struct {
  int32_t n;                /* |V| >= 0                                            */
  int64_t nnz;              /* 2|E| = row_ptr[n]                                   */
  const int64_t* row_ptr;   /* n + 1 offsets, row_ptr[0] = 0, non-decreasing        */
  const int32_t* col_idx;   /* nnz neighbour ids in [0, n)                         */
  const float* edge_len;    /* NULL: unit edges, d_ij = hop count (bytes on the device,
                               at most 255).  Else nnz positive lengths, equal on both
                               entries of an edge: d_ij = shortest-path length, summed
                               in FP32 along the path (Sec. 5.4 lays out a net with edge
                               lengths); n <= SL_WEIGHTED_MAX_N (else SL_ENOTSUP)     */
} sl_graph;

#define SL_WEIGHTED_MAX_N 16384  /* vertices of a graph with edge lengths */

typedef struct {
  int32_t dim;              /* 2 or 3                                              */
  int32_t max_iter;         /* >= 0; 0 returns X unchanged                         */
  double omega;             /* relaxation factor, finite, in (0, 16]                */
  double tol;               /* >= 0, on res_k                                     */
  int32_t safeguard;        /* 1: Alg. 2's safeguard; 0: always keep X~           */
  int32_t check_every;      /* iterations between host polls of the stop flag;
                               <= 0 selects a default from the graph size          */
  uint32_t flags;           /* SL_FLAG_*                                           */
  int32_t ordering;         /* SL_ORDER_JACOBI (default) or SL_ORDER_EXACT           */
  double* trace;            /* NULL or device buffer of max_iter * SL_TRACE_COLS
                               doubles, row k written by iteration k               */
  float* xtrace;            /* NULL or device buffer of max_iter * n * dim floats:
                               the placement after every iteration                  */
  int32_t strategy;         /* SL_OMEGA_FIXED (default), SL_OMEGA_SCHEDULE, SL_OMEGA_ENUM,
                               SL_OMEGA_AUTO                                        */
  int32_t reserved2;
  const double* omega_schedule; /* host, iter_offset + max_iter classical factors: entries
                                   iter_offset .. iter_offset + max_iter - 1 are read and
                                   must lie in (0, 16] (SL_OMEGA_SCHEDULE), else NULL */
  const float* omega_vertex;    /* NULL, or device, n classical factors in (0, 16]: vertex i
                                   extrapolates by omega_vertex[i] - 1 (SL_OMEGA_FIXED only;
                                   `omega` is then unused)                           */
  double inner_tol;         /* SL_ORDER_EXACT: relative residual of each solve, in [0, 1);
                               0 selects 1e-6                                        */
  int32_t inner_max_iter;   /* SL_ORDER_EXACT: conjugate-gradient steps per solve, >= 0;
                               0 selects 500                                         */
  int32_t reserved3;
  uint64_t seed;            /* SL_OMEGA_AUTO: seed of the roulette's generator       */
  int64_t iter_offset;      /* >= 0: global number of this call's first iteration, for
                               resuming a run from its returned placement: the factor
                               schedule and the probabilistic draws continue from there
                               (trace rows stay local: row k is iteration iter_offset + k) */
} sl_options;

typedef struct {
  int32_t iterations;       /* steps taken                                         */
  int32_t converged;        /* 1 if res <= tol was reached (or n <= 1)             */
  int32_t rejected;         /* extrapolations refused by the safeguard            */
  int32_t inner_iterations; /* SL_ORDER_EXACT: conjugate-gradient steps, summed    */
  double residual;          /* res of the last step                               */
  double stress;            /* f of the returned placement (NaN with
                               SL_FLAG_NO_FINAL_STRESS)                           */
  double plan_ms;           /* time of sl_plan_create (sl_layout: distances+weights) */
  double run_ms;            /* device time of the iteration loop                  */
  double rel_stress_drop;   /* (f(X^{K-1}) - f(X^K)) / f(X^{K-1}) over the last
                               iteration K of the call: the relative stress decrease
                               the paper's "rel err" column (Table 1) is read as; NaN
                               with SL_FLAG_NO_FINAL_STRESS, when no iteration ran or
                               f(X^{K-1}) = 0                                         */
} sl_result;

typedef struct sl_plan sl_plan;

/* Fill `opt` with defaults: dim 2, omega 1, tol 1e-3, max_iter 1000, safeguard 1,
 * everything else 0 / NULL. */
void sl_default_options(sl_options* opt);

/* Check a graph and options on the host, with no HIP call.  `opt` may be NULL
 * (graph only).  Returns SL_OK, SL_EINVAL or SL_ENOTSUP. */
sl_status sl_validate(const sl_graph* g, const sl_options* opt);

/* Build the per-graph state the iteration reads (Sec. 2): ideal distances d_ij
 * as hop counts by a multi-source breadth-first search on the device, stored
 * as bytes (0 = same vertex or no path), and the weight sums W_i = sum_j d_ij^-2
 * (the diagonal of L^W, Prop. 2.1).  `dim` (2 or 3) sizes the iterate buffers.
 * Errors: SL_EINVAL, SL_ENOTSUP, SL_ERANGE (a distance above 255), SL_ENOMEM,
 * SL_EDEVICE.  On success *out owns about n_pad^2 bytes + O(n) device memory,
 * n_pad = n rounded up to 64. */
sl_status sl_plan_create(const sl_graph* g, int32_t dim, void* stream, sl_plan** out);

/* Run Algorithm 2 from the placement in X (device, n * dim floats, row-major)
 * and write the final placement back to X.  Each iteration:
 *   1. F_i = sum_j w_ij (d_ij - r_ij) u_ij at X^k (eq. 5 residual, all pairs)
 *   2. X^H = X^k + F / W (W_i = 0: the vertex keeps its place), or with
 *      SL_ORDER_EXACT the solution of eq. 5 by conjugate gradients started
 *      from X^k (whose residual is F); res_k
 *   3. X~ = X^H + (omega - 1)(X^H - X^k)          (eq. 11)
 *   4. keep X~ iff f(X~) - f(X^H) <= 0              (Alg. 2, the safeguard)
 *   5. stop when res_k <= tol or after max_iter steps
 * `out` may be NULL.  Not converging within max_iter is not an error.
 * Edge-length plans run the Jacobi step with a fixed, scheduled or per-vertex
 * factor (SL_OMEGA_ENUM and SL_ORDER_EXACT: SL_ENOTSUP).
 * Errors: SL_EINVAL (opt, or opt->dim differs from the plan's), SL_ENUMERIC
 * (X is then the last finite iterate), SL_ENOTSUP, SL_EDEVICE. */
sl_status sl_plan_run(sl_plan* plan, float* X, const sl_options* opt, void* stream, sl_result* out);

/* f(X) of eq. 1 for a device placement X (n * dim floats), into *f (host). */
sl_status sl_plan_stress(sl_plan* plan, const float* X, int32_t dim, void* stream, double* f);

/* Copy distance rows out of a hop-count plan: out[k * n + j] = d(rows[k], j)
 * as stored (0 for j = rows[k] or no path).  `rows` and `out` are host memory.
 * SL_EINVAL for an edge-length plan. */
sl_status sl_plan_distance_rows(sl_plan* plan, const int32_t* rows, int32_t nrows, void* stream,
                                uint8_t* out);

/* The same as floats, for both kinds of plan: hop counts or path lengths
 * (0 for j = rows[k] or no path).  `rows` and `out` (nrows * n) are host memory. */
sl_status sl_plan_distance_rows_f32(sl_plan* plan, const int32_t* rows, int32_t nrows, void* stream, float* out);

/* Edge-length plans: rows of the shortest-path trees, out[k * n + v] = the
 * predecessor of v on the path from rows[k] (the lowest-numbered neighbour u
 * with d(rows[k], u) + len(u, v) = d(rows[k], v)), -1 for v = rows[k] or no
 * path.  The distance of a pair s < t is the length of the tree path of s
 * (d_ts is set to d_st).  Host memory; SL_EINVAL for hop-count plans. */
sl_status sl_plan_tree_rows(sl_plan* plan, const int32_t* rows, int32_t nrows, void* stream, int32_t* out);

/* Edge-length plans: replace the lengths (host, nnz, same graph) and rebuild
 * the distances, trees and weight sums.  Errors: SL_EINVAL (not an
 * edge-length plan, lengths invalid), SL_EDEVICE. */
sl_status sl_plan_set_lengths(sl_plan* plan, const float* edge_len, void* stream);

/* Copy the weight sums W_i (n doubles) to host memory. */
sl_status sl_plan_weights(sl_plan* plan, void* stream, double* W);

/* Measurement: device time of each kernel of one iteration, in ms, averaged
 * over `reps` back-to-back launches and timed with HIP events on the stream
 * the kernels run on (the plan's own stream, ordered after `stream`).  The
 * iteration starts from the device placement X (n * dim floats, not
 * modified) with relaxation factor `omega`:
 *   ms[0] all-pairs force pass over every ordered pair (k_force)
 *   ms[1] Jacobi update + extrapolation
 *   ms[2] safeguard pass         ms[3] select + termination test
 *   ms[4] one application of L^W (the all-pairs matvec of a conjugate-
 *         gradient step of SL_ORDER_EXACT, over unordered pairs with its
 *         reduction kernel from n_pad 24576 as the step takes it; 0 for
 *         edge-length plans)
 *   ms[5] the force pass once per unordered pair with its reduction kernel
 *         (SL_FLAG_SYM_FORCE; allocates its buffers on first use)
 *   ms[6] the force pass at X~ with the safeguard summed in (the pass that
 *         replaces ms[0] + ms[2] in an iteration that extrapolates)
 *   ms[7] the force pass over unordered pairs at X~ with the bounds of the
 *         safeguard (trace columns 5 and 6) summed in, with its reduction
 *         kernel (SL_FLAG_SYM_FORCE)
 *   ms[8] the same with f(X~) - f(X^H) itself summed in as well (the variant an
 *         iteration takes after one whose bounds left the decision open)
 * ms holds 9 doubles.
 * For profilers and benchmarks; the iterate buffers of the plan are left in an
 * unspecified state (a later sl_plan_run starts from its own X). */
sl_status sl_plan_profile(sl_plan* plan, const float* X, int32_t dim, double omega, int32_t reps, void* stream,
                          double* ms);

/* ---------------------------------------------------------------------------
 * Reverse mode (the unrolled layout as a differentiable function).
 *
 * The unrolled layout maps the initial placement X^0 and, for edge-length
 * plans, the edge lengths (through d_ij = shortest-path length) to X^K after
 * exactly K iterations of Algorithm 2 with the Jacobi step and a fixed omega.
 * Its derivative holds the safeguard decisions (Alg. 2, the safeguard) at those
 * the forward run took: they are piecewise constant in the inputs.
 * ------------------------------------------------------------------------- */

/* f(X) of eq. 1 into *f and its gradient G_i = sum_j 2 w_ij (r_ij - d_ij) u_ij
 * into G (device, n * dim floats); X is a device placement (n * dim floats). */
sl_status sl_plan_stress_grad(sl_plan* plan, const float* X, int32_t dim, void* stream, double* f, float* G);

/* Run exactly opt->max_iter = K iterations from X (device, n * dim floats, in
 * place; opt->tol is not used) and keep a tape for sl_plan_unroll_backward:
 * the placements X^{m c} (c = ckpt_every >= 1) and the decision of every
 * iteration.  The strategy must be SL_OMEGA_FIXED without per-vertex factors
 * and the ordering SL_ORDER_JACOBI (else SL_ENOTSUP); opt->trace and
 * opt->xtrace must be NULL.  A later call replaces the tape. */
sl_status sl_plan_unroll(sl_plan* plan, float* X, const sl_options* opt, int32_t ckpt_every, void* stream,
                         sl_result* out);

/* Reverse mode through the last sl_plan_unroll: given G = dL/dX^K (device,
 * n * dim floats) write dL/dX^0 into gX0 (device, n * dim floats) and, if
 * glen is not NULL (edge-length plans only), dL/dlen into glen (device, nnz
 * floats: both entries of an edge hold the edge's derivative).  Each segment
 * of c iterations is recomputed from its checkpoint.  Edge-length derivatives
 * route dL/dd_st of each pair s < t along the tree path of s (the plan's
 * trees: sl_plan_tree_rows).  Errors: SL_EINVAL (no tape, glen on a hop-count
 * plan), SL_ENOMEM, SL_EDEVICE. */
sl_status sl_plan_unroll_backward(sl_plan* plan, const float* G, float* gX0, float* glen, void* stream);

/* Release a plan and all its device memory.  NULL is accepted. */
sl_status sl_plan_destroy(sl_plan* plan);

/* ---------------------------------------------------------------------------
 * Batched layouts: many independent graphs of at most SL_BATCH_MAX_N vertices,
 * each laid out by Algorithm 2 exactly as above (same step, extrapolation,
 * safeguard and termination test, each graph stopping on its own), scheduled
 * together: one persistent launch in which each workgroup takes the next graph
 * from a queue ordered largest first and keeps its iterates in LDS.
 * ------------------------------------------------------------------------- */
#define SL_BATCH_MAX_N 1024
#define SL_BATCH_CLASSES 16   /* size classes n_pad = 64, 128, ..., 1024 */

typedef struct {
  int32_t num_graphs;        /* >= 0                                                   */
  const int64_t* graph_ptr;  /* host, num_graphs + 1 vertex offsets, graph_ptr[0] = 0: graph g
                                owns vertices graph_ptr[g] .. graph_ptr[g+1]-1 of the
                                concatenated graph; each graph has <= SL_BATCH_MAX_N vertices */
  int64_t nnz;               /* entries of the concatenated CSR                         */
  const int64_t* row_ptr;    /* host, graph_ptr[num_graphs] + 1 offsets                  */
  const int32_t* col_idx;    /* host, nnz global neighbour ids; symmetric, no self loops or
                                duplicates, and every edge stays inside its graph          */
} sl_batch;

typedef struct sl_batch_plan sl_batch_plan;

/* Distances (breadth-first search) and weight sums of every graph, on the
 * device, one workgroup per graph.  Errors: SL_EINVAL, SL_ERANGE (a distance
 * above 255 hops), SL_ENOMEM, SL_EDEVICE. */
sl_status sl_batch_plan_create(const sl_batch* b, int32_t dim, void* stream, sl_batch_plan** out);

/* Autotuner: times runs from the device placement X (not modified) for
 * workgroup sizes 256/512/1024 (whole runs with opt's tol and max_iter when
 * opt->tol > 0: a launch lasts as long as its slowest graph; else short runs)
 * and, per size class, the number of column slices of the all-pairs passes
 * (short runs: tol 0, min(opt->max_iter, 8) iterations), and keeps the
 * fastest in the plan.  config (host, may be NULL) receives
 * 1 + SL_BATCH_CLASSES ints: the workgroup size, then the slices per class
 * (0 for classes with no graph). */
sl_status sl_batch_plan_tune(sl_batch_plan* plan, const float* X, const sl_options* opt, void* stream,
                             int32_t* config);

/* Lay out every graph from the concatenated device placement X
 * (graph_ptr[num_graphs] x dim floats, row-major) in place.  opt->trace,
 * opt->xtrace and opt->omega_vertex must be NULL, the strategy fixed and the
 * ordering SL_ORDER_JACOBI (others: SL_ENOTSUP).  per_graph (host, num_graphs entries) and total may
 * be NULL; total holds the largest iteration count and residual, converged = 1
 * iff every graph converged, the sum of rejections, and run_ms. */
sl_status sl_batch_plan_run(sl_batch_plan* plan, float* X, const sl_options* opt, void* stream, sl_result* per_graph,
                            sl_result* total);

sl_status sl_batch_plan_destroy(sl_batch_plan* plan);

/* ---------------------------------------------------------------------------
 * Allocation-free batched layout, for callers that cannot allocate device
 * memory: code that must not call hipMalloc (work around HIP graph captures,
 * tight serving loops, harnesses that forbid allocation).
 *
 * The same as sl_batch_plan_create(b, opt->dim) + sl_batch_plan_run(opt) +
 * sl_batch_plan_destroy with the untuned defaults (same kernels and launch
 * shapes, so the same per-graph placements and results bit for bit), except:
 *   - No device or host allocation: the distances, weights, descriptors and
 *     the CSR copy live in the library's own device array of
 *     SL_NOALLOC_SCRATCH_BYTES, one per GPU, held from library load until the
 *     process ends; host staging is static.  A batch needs
 *       sum_g n_pad_g^2 + 8 sum_g n_pad_g + 8 (n_total + 1) + 4 nnz
 *       + 72 num_graphs bytes (n_pad_g = n_g rounded up to 64), each of its
 *     nine regions rounded up to 256 bytes; a larger batch (or more than
 *     SL_NOALLOC_SCRATCH_BYTES / 4096 graphs) returns SL_EINVAL before any
 *     device work, with the bytes needed in the message.
 *   - Everything runs on `stream`; the call synchronizes it twice (the
 *     distance check and the results).  plan_ms, run_ms and rel_stress_drop are
 *     NaN (no events are created).
 *   - Every call on a GPU shares that GPU's array, which keeps the last call's
 *     contents; the library holds a process-wide lock for the whole call, so
 *     calls from several host threads run one after another.
 * X, opt, per_graph and total as in sl_batch_plan_run.  Errors: SL_EINVAL,
 * SL_ENOTSUP, SL_ERANGE, SL_ENUMERIC, SL_EDEVICE. */
#define SL_NOALLOC_SCRATCH_BYTES (16u * 1024u * 1024u)
sl_status sl_batch_layout_noalloc(const sl_batch* b, float* X, const sl_options* opt, void* stream,
                                  sl_result* per_graph, sl_result* total);

/* layout(G, X0, omega, tol, max_iter) -> X: sl_plan_create + sl_plan_run +
 * sl_plan_destroy. */
sl_status sl_layout(const sl_graph* g, float* X, const sl_options* opt, void* stream, sl_result* out);

/* Message of the calling thread's last failed call ("" if none). */
const char* sl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SORLAYOUT_H */
