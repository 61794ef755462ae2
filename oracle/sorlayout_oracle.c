/*
 * sorlayout oracle: a plain IEEE-double reference of the SOR-accelerated
 * stress-majorization graph layout of Wang & Wang, "A Fast Successive
 * Over-Relaxation Algorithm for Force-Directed Network Graph Drawing",
 * Sci. China Inf. Sci. 55:677 (2012), arXiv:1711.01228.
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
 * CPU-baseline leg call it; the product library neither links nor calls it,
 * and the two share no code, headers or tables.
 *
 * It is slow and direct on purpose.  Each function writes out one definition
 * of the paper in the paper's notation: the stress (eq. 1), the Laplacians
 * L^W and L^Y and the majorant g (Prop. 2.1, eq. 2), the linear system of the
 * majorization step (Prop. 2.3, eq. 5), Algorithms 1 and 2 with the
 * extrapolation of eq. 10/11.  There is no blocking, fusion or reordering.
 * OpenMP only hands independent rows or sources to threads; every sum that
 * crosses rows is taken serially in index order, so results do not depend on
 * the thread count.
 *
 * Conventions
 *   vertices     0 .. n-1 (the paper numbers them 1 .. n)
 *   X            row-major n x dim, dim >= 1
 *   D            row-major n x n ideal distances, D[i][i] = 0, +INFINITY for
 *                a pair in different components
 *   w_ij         d_ij^-2 for 0 < d_ij < inf, else 0 (Sec. 5.1 takes w = d^-2;
 *                a pair with no path contributes nothing, the limit d -> inf)
 *   CSR graph    symmetric, row_ptr[n+1] (int64), col_idx[nnz] (int32),
 *                optional positive edge lengths len[nnz]
 *
 * Compiled with -O2 -ffp-contract=off and no fast-math: IEEE sqrt and divide.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SLO_OK 0
#define SLO_EINVAL (-1)
#define SLO_ENOMEM (-2)
#define SLO_ENUMERIC (-5)

enum { SLO_JACOBI = 0, SLO_EXACT = 1, SLO_GAUSS_SEIDEL = 2 };

/* ---------------------------------------------------------------------- */
/* Weights w_ij = d_ij^-2 (Sec. 5.1), the products that appear in L^Y      */
/* (w_ij d_ij) and in the constant C of eq. 2 (w_ij d_ij^2).              */
/* ---------------------------------------------------------------------- */
static double w_of(double d) { return (d > 0.0 && isfinite(d)) ? 1.0 / (d * d) : 0.0; }
static double wd_of(double d) { return (d > 0.0 && isfinite(d)) ? 1.0 / d : 0.0; }
static double wdd_of(double d) { return (d > 0.0 && isfinite(d)) ? 1.0 : 0.0; }

static double dist(int dim, const double* a, const double* b) {
  double s = 0.0;
  for (int c = 0; c < dim; ++c) {
    double t = a[c] - b[c];
    s += t * t;
  }
  return sqrt(s);
}

/* ---------------------------------------------------------------------- */
/* Ideal distances d_ij: graph-theoretic shortest paths.  Hop counts when  */
/* len == NULL (breadth-first search); sums of edge lengths otherwise      */
/* (Dijkstra with a binary heap), as for the weighted railway net of Sec. 5.4. */
/* ---------------------------------------------------------------------- */
typedef struct { double key; int32_t v; } heap_item;

static void heap_push(heap_item* h, int64_t* size, double key, int32_t v) {
  int64_t i = (*size)++;
  h[i].key = key;
  h[i].v = v;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h[p].key <= h[i].key) break;
    heap_item t = h[p]; h[p] = h[i]; h[i] = t;
    i = p;
  }
}

static heap_item heap_pop(heap_item* h, int64_t* size) {
  heap_item top = h[0];
  h[0] = h[--(*size)];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, m = i;
    if (l < *size && h[l].key < h[m].key) m = l;
    if (r < *size && h[r].key < h[m].key) m = r;
    if (m == i) break;
    heap_item t = h[m]; h[m] = h[i]; h[i] = t;
    i = m;
  }
  return top;
}

int slo_sssp(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* len,
             int32_t src, double* drow) {
  if (n < 0 || src < 0 || src >= n) return SLO_EINVAL;
  for (int32_t v = 0; v < n; ++v) drow[v] = INFINITY;
  drow[src] = 0.0;
  if (len == NULL) {
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!queue) return SLO_ENOMEM;
    int32_t head = 0, tail = 0;
    queue[tail++] = src;
    while (head < tail) {
      int32_t u = queue[head++];
      for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
        int32_t v = col_idx[e];
        if (isinf(drow[v])) {
          drow[v] = drow[u] + 1.0;
          queue[tail++] = v;
        }
      }
    }
    free(queue);
    return SLO_OK;
  }
  int64_t nnz = row_ptr[n];
  heap_item* heap = (heap_item*)malloc(sizeof(heap_item) * (size_t)(nnz + 1));
  char* done = (char*)calloc((size_t)(n > 0 ? n : 1), 1);
  if (!heap || !done) { free(heap); free(done); return SLO_ENOMEM; }
  int64_t size = 0;
  heap_push(heap, &size, 0.0, src);
  while (size > 0) {
    heap_item it = heap_pop(heap, &size);
    int32_t u = it.v;
    if (done[u]) continue;
    done[u] = 1;
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      int32_t v = col_idx[e];
      double nd = drow[u] + len[e];
      if (nd < drow[v]) {
        drow[v] = nd;
        heap_push(heap, &size, nd, v);
      }
    }
  }
  free(heap);
  free(done);
  return SLO_OK;
}

int slo_apsp(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* len, double* D) {
  int status = SLO_OK;
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t s = 0; s < n; ++s) {
    int r = slo_sssp(n, row_ptr, col_idx, len, s, D + (size_t)s * n);
    if (r != SLO_OK) {
#pragma omp critical
      status = r;
    }
  }
  return status;
}

/* Distances from a list of sources: rows[k] -> Drows[k][0..n). */
int slo_sssp_rows(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* len,
                  const int32_t* rows, int32_t nrows, double* Drows) {
  int status = SLO_OK;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t k = 0; k < nrows; ++k) {
    int r = slo_sssp(n, row_ptr, col_idx, len, rows[k], Drows + (size_t)k * n);
    if (r != SLO_OK) {
#pragma omp critical
      status = r;
    }
  }
  return status;
}

/* W_i = sum_{j != i} w_ij: the diagonal of L^W (Prop. 2.1). */
void slo_weight_sums(int32_t n, const double* D, double* W) {
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int32_t j = 0; j < n; ++j)
      if (j != i) s += w_of(D[(size_t)i * n + j]);
    W[i] = s;
  }
}

/* ---------------------------------------------------------------------- */
/* Stress, eq. 1: f(X) = sum_{i<j} w_ij (||x_i - x_j|| - d_ij)^2.          */
/* ---------------------------------------------------------------------- */
double slo_stress(int32_t n, int32_t dim, const double* D, const double* X) {
  double* part = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  if (!part) return NAN;
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int32_t j = i + 1; j < n; ++j) {
      double d = D[(size_t)i * n + j];
      double w = w_of(d);
      if (w == 0.0) continue;
      double e = dist(dim, X + (size_t)i * dim, X + (size_t)j * dim) - d;
      s += w * e * e;
    }
    part[i] = s;
  }
  double f = 0.0;
  for (int32_t i = 0; i < n; ++i) f += part[i];
  free(part);
  return f;
}

/* f(XA) - f(XB), summed pair by pair as sum_{i<j} [w(rA-d)^2 - w(rB-d)^2],
 * plus the scale sum_{i<j} |w(rA-d)^2 - w(rB-d)^2| of that sum: the
 * safeguard comparison of Algorithm 2 and the size of the terms it rests on.
 * Row i's share (pairs j > i) from its distance row drow. */
static void stress_delta_row(int32_t n, int32_t dim, const double* drow, int32_t i, const double* XA,
                             const double* XB, double* sd_out, double* ss_out) {
  double sd = 0.0, ss = 0.0;
  for (int32_t j = i + 1; j < n; ++j) {
    double d = drow[j];
    double w = w_of(d);
    if (w == 0.0) continue;
    double ea = dist(dim, XA + (size_t)i * dim, XA + (size_t)j * dim) - d;
    double eb = dist(dim, XB + (size_t)i * dim, XB + (size_t)j * dim) - d;
    double t = w * ea * ea - w * eb * eb;
    sd += t;
    ss += fabs(t);
  }
  *sd_out = sd;
  *ss_out = ss;
}

void slo_stress_delta(int32_t n, int32_t dim, const double* D, const double* XA, const double* XB,
                      double* delta, double* scale) {
  double* pd = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double* ps = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  if (!pd || !ps) { free(pd); free(ps); *delta = NAN; *scale = NAN; return; }
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t i = 0; i < n; ++i) stress_delta_row(n, dim, D + (size_t)i * n, i, XA, XB, pd + i, ps + i);
  double a = 0.0, b = 0.0;
  for (int32_t i = 0; i < n; ++i) { a += pd[i]; b += ps[i]; }
  *delta = a;
  *scale = b;
  free(pd);
  free(ps);
}

/* Bounds of the safeguard's sum f(XA) - f(XB) from first-order terms.   */
/* With t = xA_i - xA_j, rA = |t|, rB = |xB_i - xB_j|, e = (xA_i - xB_i)  */
/* - (xA_j - xB_j), m = rA^2 - rB^2, c = 1/(d rA) - 1/d^2 (the pair's     */
/* coefficient in the eq. 5 residual at XA), kappa = 1/(d rA) and        */
/* delta = rA - rB, each pair's term of eq. 1's difference is             */
/*   w (rA - d)^2 - w (rB - d)^2 = w m - (2/d) delta = -c m - kappa delta^2 */
/* (m = delta (2 rA - delta)), and 0 <= delta^2 <= |e|^2 (triangle        */
/* inequality).  So U = sum -c m >= f(XA) - f(XB) >= U - sum kappa |e|^2 = L. */
/* out = {U, L, sum |c m|, sum kappa |e|^2}; U = +inf when two vertices   */
/* with a path between them coincide in XA (c is unbounded there).        */
/* Test infrastructure for the bounds the GPU's unordered pass reports;   */
/* the method's own decision is slo_stress_delta's.                       */
static void stress_bounds_row(int32_t n, int32_t dim, const double* drow, int32_t i, const double* XA,
                              const double* XB, double out[4]) {
  double u = 0.0, q = 0.0, su = 0.0;
  for (int32_t j = i + 1; j < n; ++j) {
    const double d = drow[j];
    const double w = w_of(d);
    if (w == 0.0) continue;
    const double ra = dist(dim, XA + (size_t)i * dim, XA + (size_t)j * dim);
    const double rb = dist(dim, XB + (size_t)i * dim, XB + (size_t)j * dim);
    double e2 = 0.0;
    for (int32_t k = 0; k < dim; ++k) {
      const double e = (XA[(size_t)i * dim + k] - XB[(size_t)i * dim + k]) -
                       (XA[(size_t)j * dim + k] - XB[(size_t)j * dim + k]);
      e2 += e * e;
    }
    if (ra == 0.0) {
      u = INFINITY;
      continue;
    }
    const double kappa = 1.0 / (d * ra);
    const double c = kappa - w;
    const double m = ra * ra - rb * rb;
    u += -c * m;
    su += fabs(c * m);
    q += kappa * e2;
  }
  out[0] = u;
  out[1] = u - q;
  out[2] = su;
  out[3] = q;
}

void slo_stress_delta_bounds(int32_t n, int32_t dim, const double* D, const double* XA, const double* XB,
                             double out[4]) {
  double* part = (double*)malloc(sizeof(double) * 4 * (size_t)(n > 0 ? n : 1));
  if (!part) { for (int k = 0; k < 4; ++k) out[k] = NAN; return; }
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t i = 0; i < n; ++i) stress_bounds_row(n, dim, D + (size_t)i * n, i, XA, XB, part + 4 * (size_t)i);
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  for (int32_t i = 0; i < n; ++i)
    for (int k = 0; k < 4; ++k) t[k] += part[4 * (size_t)i + k];
  t[1] = t[0] - t[3];  /* L as U - sum kappa |e|^2 of the totals */
  for (int k = 0; k < 4; ++k) out[k] = t[k];
  free(part);
}

/* ---------------------------------------------------------------------- */
/* Laplacians of Prop. 2.1, applied to a placement.                       */
/*   l^W_ij = -w_ij (i != j),  l^W_ii = -sum_{k != i} l^W_ik              */
/*   l^Y_ij = 0 if y_i = y_j, else -w_ij d_ij / ||y_i - y_j|| (i != j),   */
/*   l^Y_ii = -sum_{k != i} l^Y_ik                                        */
/* ---------------------------------------------------------------------- */
static double lw_entry(int32_t n, const double* D, int32_t i, int32_t j) {
  if (i != j) return -w_of(D[(size_t)i * n + j]);
  double s = 0.0;
  for (int32_t k = 0; k < n; ++k)
    if (k != i) s += w_of(D[(size_t)i * n + k]);
  return s;
}

static double ly_offdiag(int32_t n, int32_t dim, const double* D, const double* Y, int32_t i, int32_t j) {
  double r = dist(dim, Y + (size_t)i * dim, Y + (size_t)j * dim);
  if (r == 0.0) return 0.0;
  return -wd_of(D[(size_t)i * n + j]) / r;
}

/* out = L^W X (n x dim) */
void slo_apply_LW(int32_t n, int32_t dim, const double* D, const double* X, double* out) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t c = 0; c < dim; ++c) {
      double s = 0.0;
      for (int32_t j = 0; j < n; ++j) s += lw_entry(n, D, i, j) * X[(size_t)j * dim + c];
      out[(size_t)i * dim + c] = s;
    }
  }
}

/* out = L^Y Y (n x dim) */
void slo_apply_LY(int32_t n, int32_t dim, const double* D, const double* Y, double* out) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t i = 0; i < n; ++i) {
    double diag = 0.0;
    for (int32_t k = 0; k < n; ++k)
      if (k != i) diag -= ly_offdiag(n, dim, D, Y, i, k);
    for (int32_t c = 0; c < dim; ++c) {
      double s = diag * Y[(size_t)i * dim + c];
      for (int32_t j = 0; j < n; ++j)
        if (j != i) s += ly_offdiag(n, dim, D, Y, i, j) * Y[(size_t)j * dim + c];
      out[(size_t)i * dim + c] = s;
    }
  }
}

/* g(X, Y) = tr(X^T L^W X) - 2 tr(X^T L^Y Y) + C, C = sum_{i<j} w_ij d_ij^2 (eq. 2). */
double slo_majorant(int32_t n, int32_t dim, const double* D, const double* X, const double* Y) {
  size_t nd = (size_t)n * dim;
  double* LX = (double*)malloc(sizeof(double) * (nd ? nd : 1));
  double* LYY = (double*)malloc(sizeof(double) * (nd ? nd : 1));
  if (!LX || !LYY) { free(LX); free(LYY); return NAN; }
  slo_apply_LW(n, dim, D, X, LX);
  slo_apply_LY(n, dim, D, Y, LYY);
  double t1 = 0.0, t2 = 0.0, C = 0.0;
  for (size_t k = 0; k < nd; ++k) {
    t1 += X[k] * LX[k];
    t2 += X[k] * LYY[k];
  }
  for (int32_t i = 0; i < n; ++i)
    for (int32_t j = i + 1; j < n; ++j) C += wdd_of(D[(size_t)i * n + j]);
  free(LX);
  free(LYY);
  return t1 - 2.0 * t2 + C;
}

/* ---------------------------------------------------------------------- */
/* The majorization step H of Algorithm 1/2: X^H solves                   */
/*   L^W X^H = L^X X          (eq. 5 with Y = X, one column per dimension) */
/* ---------------------------------------------------------------------- */

/* One Jacobi update of row i of eq. 5 from the iterate X:
 *   l^W_ii x_i^H = (L^X X)_i - sum_{j != i} l^W_ij x_j
 *   x_i^H = [ (L^X X)_i + sum_{j != i} w_ij x_j ] / W_i,
 * with (L^X X)_i = sum_{j != i, x_j != x_i} w_ij d_ij (x_i - x_j) / ||x_i - x_j||.
 * A vertex with W_i = 0 (no path to any other vertex) keeps its position. */
void slo_h_jacobi_row(int32_t n, int32_t dim, const double* drow, int32_t i, const double* X,
                      double* xh) {
  const double* xi = X + (size_t)i * dim;
  double Wi = 0.0;
  for (int32_t j = 0; j < n; ++j)
    if (j != i) Wi += w_of(drow[j]);
  if (Wi == 0.0) {
    for (int32_t c = 0; c < dim; ++c) xh[c] = xi[c];
    return;
  }
  for (int32_t c = 0; c < dim; ++c) {
    double lyx = 0.0, wx = 0.0;
    for (int32_t j = 0; j < n; ++j) {
      if (j == i) continue;
      const double* xj = X + (size_t)j * dim;
      double w = w_of(drow[j]);
      if (w == 0.0) continue;
      double r = dist(dim, xi, xj);
      if (r != 0.0) lyx += wd_of(drow[j]) / r * (xi[c] - xj[c]);
      wx += w * xj[c];
    }
    xh[c] = (lyx + wx) / Wi;
  }
}

void slo_h_jacobi(int32_t n, int32_t dim, const double* D, const double* X, double* XH) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t i = 0; i < n; ++i) slo_h_jacobi_row(n, dim, D + (size_t)i * n, i, X, XH + (size_t)i * dim);
}

/* Jacobi rows for a sample of vertices whose distance rows are given:
 * Drows[k] is the distance row of vertex rows[k]; XH_rows[k] receives x^H of it. */
void slo_h_jacobi_rows(int32_t n, int32_t dim, const double* Drows, const int32_t* rows, int32_t nrows,
                       const double* X, double* XH_rows) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t k = 0; k < nrows; ++k)
    slo_h_jacobi_row(n, dim, Drows + (size_t)k * n, rows[k], X, XH_rows + (size_t)k * dim);
}

/* Sequential (Gauss-Seidel) sweep of the same row update: rows are updated
 * in place for i = 0 .. n-1, each one seeing the newest positions of the rows
 * before it (the "one-by-one" vertex update of Kamada-Kawai style methods). */
void slo_h_gauss_seidel(int32_t n, int32_t dim, const double* D, const double* X, double* XH) {
  memcpy(XH, X, sizeof(double) * (size_t)n * dim);
  double* tmp = (double*)malloc(sizeof(double) * (size_t)(dim > 0 ? dim : 1));
  if (!tmp) return;
  for (int32_t i = 0; i < n; ++i) {
    slo_h_jacobi_row(n, dim, D + (size_t)i * n, i, XH, tmp);
    for (int32_t c = 0; c < dim; ++c) XH[(size_t)i * dim + c] = tmp[c];
  }
  free(tmp);
}

/* Exact solve of eq. 5, as the paper reduces it: within each connected
 * component the lowest-numbered vertex p is held fixed, its row and column
 * are dropped, and the remaining symmetric positive definite system is
 * solved by a Cholesky factorization computed once.  The paper fixes
 * x_1 = 0; holding x_p at its current position instead only translates the
 * component. */
typedef struct {
  int32_t n;
  int32_t ncomp;
  int32_t* comp_start;  /* ncomp + 1 offsets into verts */
  int32_t* verts;       /* vertices grouped by component, ascending; first = pinned */
  double** chol;        /* per component: lower factor of size (m x m), m = size - 1 */
} slo_exact_ctx;

void slo_exact_free(slo_exact_ctx* ctx) {
  if (!ctx) return;
  if (ctx->chol)
    for (int32_t c = 0; c < ctx->ncomp; ++c) free(ctx->chol[c]);
  free(ctx->chol);
  free(ctx->comp_start);
  free(ctx->verts);
  free(ctx);
}

slo_exact_ctx* slo_exact_prepare(int32_t n, const double* D) {
  slo_exact_ctx* ctx = (slo_exact_ctx*)calloc(1, sizeof(slo_exact_ctx));
  if (!ctx) return NULL;
  ctx->n = n;
  int32_t* label = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  ctx->verts = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  ctx->comp_start = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  if (!label || !ctx->verts || !ctx->comp_start) { free(label); slo_exact_free(ctx); return NULL; }
  for (int32_t i = 0; i < n; ++i) label[i] = -1;
  int32_t ncomp = 0, pos = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (label[i] >= 0) continue;
    ctx->comp_start[ncomp] = pos;
    for (int32_t j = i; j < n; ++j)
      if (label[j] < 0 && isfinite(D[(size_t)i * n + j])) {
        label[j] = ncomp;
        ctx->verts[pos++] = j;
      }
    ++ncomp;
  }
  ctx->comp_start[ncomp] = pos;
  ctx->ncomp = ncomp;
  free(label);
  ctx->chol = (double**)calloc((size_t)(ncomp > 0 ? ncomp : 1), sizeof(double*));
  if (!ctx->chol) { slo_exact_free(ctx); return NULL; }
  for (int32_t c = 0; c < ncomp; ++c) {
    int32_t s = ctx->comp_start[c], m = ctx->comp_start[c + 1] - s - 1;
    if (m <= 0) continue;
    const int32_t* v = ctx->verts + s + 1;
    double* L = (double*)calloc((size_t)m * m, sizeof(double));
    if (!L) { slo_exact_free(ctx); return NULL; }
    for (int32_t a = 0; a < m; ++a)
      for (int32_t b = 0; b < m; ++b) L[(size_t)a * m + b] = lw_entry(n, D, v[a], v[b]);
    /* in-place Cholesky, lower triangle: A = L L^T */
    for (int32_t j = 0; j < m; ++j) {
      double s2 = L[(size_t)j * m + j];
      for (int32_t k = 0; k < j; ++k) s2 -= L[(size_t)j * m + k] * L[(size_t)j * m + k];
      if (!(s2 > 0.0)) { free(L); slo_exact_free(ctx); return NULL; }
      double ljj = sqrt(s2);
      L[(size_t)j * m + j] = ljj;
#pragma omp parallel for schedule(static)
      for (int32_t i = j + 1; i < m; ++i) {
        double t = L[(size_t)i * m + j];
        for (int32_t k = 0; k < j; ++k) t -= L[(size_t)i * m + k] * L[(size_t)j * m + k];
        L[(size_t)i * m + j] = t / ljj;
      }
    }
    ctx->chol[c] = L;
  }
  return ctx;
}

int slo_h_exact(const slo_exact_ctx* ctx, int32_t dim, const double* D, const double* X, double* XH) {
  int32_t n = ctx->n;
  size_t nd = (size_t)n * dim;
  double* LYX = (double*)malloc(sizeof(double) * (nd ? nd : 1));
  if (!LYX) return SLO_ENOMEM;
  slo_apply_LY(n, dim, D, X, LYX);
  memcpy(XH, X, sizeof(double) * nd);
  for (int32_t c = 0; c < ctx->ncomp; ++c) {
    int32_t s = ctx->comp_start[c], m = ctx->comp_start[c + 1] - s - 1;
    if (m <= 0) continue;
    int32_t p = ctx->verts[s];
    const int32_t* v = ctx->verts + s + 1;
    const double* L = ctx->chol[c];
    double* y = (double*)malloc(sizeof(double) * (size_t)m);
    if (!y) { free(LYX); return SLO_ENOMEM; }
    for (int32_t col = 0; col < dim; ++col) {
      /* right-hand side: (L^X X)_i - l^W_ip x_p for the kept rows */
      for (int32_t a = 0; a < m; ++a)
        y[a] = LYX[(size_t)v[a] * dim + col] - lw_entry(n, D, v[a], p) * X[(size_t)p * dim + col];
      for (int32_t a = 0; a < m; ++a) { /* forward: L z = b */
        double t = y[a];
        for (int32_t k = 0; k < a; ++k) t -= L[(size_t)a * m + k] * y[k];
        y[a] = t / L[(size_t)a * m + a];
      }
      for (int32_t a = m - 1; a >= 0; --a) { /* backward: L^T x = z */
        double t = y[a];
        for (int32_t k = a + 1; k < m; ++k) t -= L[(size_t)k * m + a] * y[k];
        y[a] = t / L[(size_t)a * m + a];
      }
      for (int32_t a = 0; a < m; ++a) XH[(size_t)v[a] * dim + col] = y[a];
    }
    free(y);
  }
  free(LYX);
  return SLO_OK;
}

/* ---------------------------------------------------------------------- */
/* Termination measure: the relative size of the step H(X) - X,            */
/*   res = ||X^H - X||_F / ||X^H - mean(X^H)||_F   (0 when both are 0).     */
/* ---------------------------------------------------------------------- */
double slo_residual(int32_t n, int32_t dim, const double* X, const double* XH) {
  double num = 0.0, den = 0.0;
  for (int32_t c = 0; c < dim; ++c) {
    double mean = 0.0;
    for (int32_t i = 0; i < n; ++i) mean += XH[(size_t)i * dim + c];
    mean /= (n > 0 ? n : 1);
    for (int32_t i = 0; i < n; ++i) {
      double a = XH[(size_t)i * dim + c] - X[(size_t)i * dim + c];
      double b = XH[(size_t)i * dim + c] - mean;
      num += a * a;
      den += b * b;
    }
  }
  if (num == 0.0) return 0.0;
  return sqrt(num) / sqrt(den);
}

/* ---------------------------------------------------------------------- */
/* Algorithm 2 (Algorithm 1 when omega = 1).                               */
/* omega is the classical relaxation factor: the paper's factor is          */
/* omega - 1, so the extrapolation of eq. 11 reads                          */
/*   X~ = X^H + (omega - 1)(X^H - X).                                       */
/* Relaxation strategies of Sec. 5.2:                                        */
/*   fixed           one omega for every iteration                          */
/*   schedule        omega_schedule[k] at iteration k (the probabilistic     */
/*                   strategy draws this sequence by roulette; the draws are */
/*                   an input here)                                          */
/*   enumerating     the paper's factor chosen each iteration as the argmin  */
/*                   of f(X^H + c (X^H - X)) over c in {0, 0.5, ..., 9}       */
/*   per vertex      x~_i = x^H_i + (omega_i - 1)(x^H_i - x_i) (Sec. 6, (1)) */
/* ---------------------------------------------------------------------- */
typedef struct {
  int32_t iterations;
  int32_t converged;
  int32_t rejected;
  int32_t status;
  double residual;  /* residual of the last step taken */
} slo_result;

/* trace (optional): max_iter rows of SLO_TRACE_COLS doubles:
 *   [0] res_k   [1] accepted (1/0; -1 when no extrapolation is formed)
 *   [2] f(X~) - f(X^H) of the placement considered   [3] scale of that sum
 *   [4] f(X^k) (NAN unless trace_stress)
 *   [5] the paper's relaxation factor used (omega - 1; NAN for per-vertex)
 *   [6] enumerating: smallest |f-difference| between the best candidate and
 *       any other one   [7] enumerating: the larger term scale of that pair
 * xtrace (optional): max_iter placements X^{k+1}, n*dim each. */
#define SLO_TRACE_COLS 8
#define SLO_ENUM_CANDIDATES 19

int slo_layout(int32_t n, int32_t dim, const double* D, double* X, double omega, double tol,
               int32_t max_iter, int32_t ordering, int32_t safeguard, int32_t trace_stress,
               const double* omega_schedule, const double* omega_vertex, int32_t enumerate,
               double* trace, double* xtrace, slo_result* out) {
  memset(out, 0, sizeof(*out));
  if (n < 0 || dim < 1 || !(omega > 0.0) || !(tol >= 0.0) || max_iter < 0) return SLO_EINVAL;
  if (ordering != SLO_JACOBI && ordering != SLO_EXACT && ordering != SLO_GAUSS_SEIDEL) return SLO_EINVAL;
  size_t nd = (size_t)n * dim;
  double* XH = (double*)malloc(sizeof(double) * (nd ? nd : 1));
  double* XT = (double*)malloc(sizeof(double) * (nd ? nd : 1));
  slo_exact_ctx* ctx = NULL;
  if (!XH || !XT) { free(XH); free(XT); return SLO_ENOMEM; }
  if (ordering == SLO_EXACT && n > 0) {
    ctx = slo_exact_prepare(n, D);
    if (!ctx) { free(XH); free(XT); return SLO_ENOMEM; }
  }
  int status = SLO_OK;
  /* a single vertex (or none) is already laid out: no step is taken */
  for (int32_t k = 0; k < max_iter && n > 1; ++k) {
    double f_k = trace_stress ? slo_stress(n, dim, D, X) : NAN;
    /* step H: X^{k+1} <- H(X^k) */
    if (ordering == SLO_JACOBI) slo_h_jacobi(n, dim, D, X, XH);
    else if (ordering == SLO_GAUSS_SEIDEL) slo_h_gauss_seidel(n, dim, D, X, XH);
    else status = slo_h_exact(ctx, dim, D, X, XH);
    if (status != SLO_OK) break;
    for (size_t q = 0; q < nd; ++q)
      if (!isfinite(XH[q])) status = SLO_ENUMERIC;
    if (status != SLO_OK) break;
    double res = slo_residual(n, dim, X, XH);
    double accepted = -1.0, df = 0.0, scale = 0.0, used = NAN, gap = NAN, gscale = NAN;
    if (enumerate) {
      /* Sec. 5.2, enumerating strategy: c = 0 is X^H itself (difference 0) */
      double best_df = 0.0, best_scale = 0.0, best_c = 0.0;
      double dfs[SLO_ENUM_CANDIDATES], scs[SLO_ENUM_CANDIDATES];
      dfs[0] = 0.0;
      scs[0] = 0.0;
      for (int c = 1; c < SLO_ENUM_CANDIDATES; ++c) {
        const double wc = 0.5 * c;
        for (size_t q = 0; q < nd; ++q) XT[q] = XH[q] + wc * (XH[q] - X[q]);
        slo_stress_delta(n, dim, D, XT, XH, &dfs[c], &scs[c]);
        if (dfs[c] < best_df) {
          best_df = dfs[c];
          best_scale = scs[c];
          best_c = wc;
        }
      }
      gap = INFINITY;
      gscale = 0.0;
      for (int c = 0; c < SLO_ENUM_CANDIDATES; ++c) {
        if (0.5 * c == best_c) continue;
        const double gp = fabs(dfs[c] - best_df);
        if (gp < gap) {
          gap = gp;
          gscale = fmax(scs[c], best_scale);
        }
      }
      df = best_df;
      scale = best_scale;
      used = best_c;
      accepted = best_c > 0.0 ? 1.0 : 0.0;
      if (best_c == 0.0) {
        out->rejected += 1;
        memcpy(X, XH, sizeof(double) * nd);
      } else {
        for (size_t q = 0; q < nd; ++q) X[q] = XH[q] + best_c * (XH[q] - X[q]);
      }
    } else {
      const double omega_k = omega_schedule ? omega_schedule[k] : omega;
      const double omega_p = omega_k - 1.0;
      used = omega_vertex ? NAN : omega_p;
      if (omega_p == 0.0 && !omega_vertex) {
        memcpy(X, XH, sizeof(double) * nd);
      } else {
        /* extrapolation (eq. 11): X~ = X^H + omega_p (X^H - X^k), per vertex if given */
        for (int32_t i = 0; i < n; ++i) {
          const double wp = omega_vertex ? omega_vertex[i] - 1.0 : omega_p;
          for (int32_t c = 0; c < dim; ++c) {
            const size_t q = (size_t)i * dim + c;
            XT[q] = XH[q] + wp * (XH[q] - X[q]);
          }
        }
        int take = 1;
        if (safeguard) {
          /* safeguard: keep X~ only if f(X~) <= f(X^H) */
          slo_stress_delta(n, dim, D, XT, XH, &df, &scale);
          take = (df <= 0.0);
        }
        accepted = take ? 1.0 : 0.0;
        if (!take) out->rejected += 1;
        memcpy(X, take ? XT : XH, sizeof(double) * nd);
      }
    }
    out->iterations = k + 1;
    out->residual = res;
    if (trace) {
      double* row = trace + (size_t)k * SLO_TRACE_COLS;
      row[0] = res;
      row[1] = accepted;
      row[2] = df;
      row[3] = scale;
      row[4] = f_k;
      row[5] = used;
      row[6] = gap;
      row[7] = gscale;
    }
    if (xtrace) memcpy(xtrace + (size_t)k * nd, X, sizeof(double) * nd);
    if (res <= tol) {
      out->converged = 1;
      break;
    }
  }
  if (n <= 1 && status == SLO_OK) out->converged = 1;
  slo_exact_free(ctx);
  free(XH);
  free(XT);
  out->status = status;
  return status;
}

/* ====================================================================== */
/* Derivatives (reverse mode) of the unrolled Jacobi-SOR iteration.       */
/* ====================================================================== */

/* Shortest-path tree of source src for positive edge lengths: drow as
 * slo_sssp computes it (Dijkstra), pred[v] = the lowest-numbered neighbour u
 * with drow[u] + len(u, v) == drow[v] (ties broken by the lowest id), -1 for
 * src and for vertices with no path.  Lengths must be symmetric. */
int slo_sp_tree(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* len, int32_t src,
                double* drow, int32_t* pred) {
  int r = slo_sssp(n, row_ptr, col_idx, len, src, drow);
  if (r != SLO_OK) return r;
  for (int32_t v = 0; v < n; ++v) {
    pred[v] = -1;
    if (v == src || isinf(drow[v])) continue;
    for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      int32_t u = col_idx[e];
      double l = len ? len[e] : 1.0;
      if (drow[u] + l == drow[v] && (pred[v] < 0 || u < pred[v])) pred[v] = u;
    }
  }
  return SLO_OK;
}

int slo_sp_trees(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* len, double* D,
                 int32_t* P) {
  int status = SLO_OK;
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t s = 0; s < n; ++s) {
    int r = slo_sp_tree(n, row_ptr, col_idx, len, s, D + (size_t)s * n, P + (size_t)s * n);
    if (r != SLO_OK) {
#pragma omp critical
      status = r;
    }
  }
  return status;
}

/* Gradient of the stress (eq. 1): G_i = sum_{j != i} 2 w_ij (r_ij - d_ij) u_ij,
 * u_ij = (x_i - x_j) / r_ij (pairs with r_ij = 0 contribute 0). */
void slo_stress_grad(int32_t n, int32_t dim, const double* D, const double* X, double* G) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t c = 0; c < dim; ++c) G[(size_t)i * dim + c] = 0.0;
    for (int32_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double d = D[(size_t)i * n + j];
      double w = w_of(d);
      double r = dist(dim, X + (size_t)i * dim, X + (size_t)j * dim);
      if (w == 0.0 || r == 0.0) continue;
      for (int32_t c = 0; c < dim; ++c)
        G[(size_t)i * dim + c] += 2.0 * w * (r - d) * (X[(size_t)i * dim + c] - X[(size_t)j * dim + c]) / r;
    }
  }
}

/* Reverse mode through K iterations of Algorithm 2 with the Jacobi step and
 * a fixed omega, the safeguard decisions held at acc[k] (1: X~ kept, else
 * X^H kept; as the trace column of slo_layout records them).
 *
 * Forward, row form of eq. 5 (one sweep, the other vertices at X):
 *   x^H_i = (1/W_i) [ sum_j w_ij x_j + sum_j (1/d_ij) u_ij ],  W_i = sum_j w_ij,
 *   X^{k+1} = a X^H - b X,   (a, b) = (omega, omega - 1) if acc[k] = 1, else (1, 0).
 * Backward, with h = dL/dX^H = a Gbar and g_i = h_i / W_i:
 *   dx^H_i/dx_i = (1/W_i) sum_j P_ij,  dx^H_i/dx_j = (1/W_i) (w_ij I - P_ij),
 *   P_ij = (1/(d_ij r_ij)) (I - u_ij u_ij^T),
 *   dL/dx_m = sum_j P_mj (g_m - g_j) + sum_j w_mj g_j - b Gbar_m,
 *   dL/dd_ij (row i's use of d_ij) += g_i . [ -2 w_ij (1/d_ij) (x_j - x^H_i) - w_ij u_ij ].
 * A vertex with W_i = 0 keeps its place: dL/dx_i gets h_i.
 * Outputs: gX0 = dL/dX^0 (n x dim), gD (n x n) = dL/dd with d_ij and d_ji one
 * variable (gD[i][j] = gD[j][i] = the two row uses summed). */
int slo_layout_vjp(int32_t n, int32_t dim, const double* D, const double* X0, double omega, int32_t K,
                   const double* acc, const double* G, double* gX0, double* gD) {
  size_t nd = (size_t)n * dim;
  double* Xs = (double*)malloc(sizeof(double) * nd * (size_t)(K + 1));
  double* XHs = (double*)malloc(sizeof(double) * nd * (size_t)(K > 0 ? K : 1));
  double* W = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double* gb = (double*)malloc(sizeof(double) * (nd ? nd : 1));
  double* gw = (double*)malloc(sizeof(double) * (nd ? nd : 1));
  double* gn = (double*)malloc(sizeof(double) * (nd ? nd : 1));
  if (!Xs || !XHs || !W || !gb || !gw || !gn) {
    free(Xs); free(XHs); free(W); free(gb); free(gw); free(gn);
    return SLO_ENOMEM;
  }
  slo_weight_sums(n, D, W);
  memcpy(Xs, X0, sizeof(double) * nd);
  for (int32_t k = 0; k < K; ++k) {
    const double* X = Xs + (size_t)k * nd;
    double* XH = XHs + (size_t)k * nd;
    double* Xn = Xs + (size_t)(k + 1) * nd;
    slo_h_jacobi(n, dim, D, X, XH);
    double a = acc[k] == 1.0 ? omega : 1.0, b = acc[k] == 1.0 ? omega - 1.0 : 0.0;
    for (size_t q = 0; q < nd; ++q) Xn[q] = a * XH[q] - b * X[q];
  }
  memcpy(gb, G, sizeof(double) * nd);
  memset(gD, 0, sizeof(double) * (size_t)n * n);
  for (int32_t k = K - 1; k >= 0; --k) {
    const double* X = Xs + (size_t)k * nd;
    const double* XH = XHs + (size_t)k * nd;
    double a = acc[k] == 1.0 ? omega : 1.0, b = acc[k] == 1.0 ? omega - 1.0 : 0.0;
    for (int32_t i = 0; i < n; ++i)
      for (int32_t c = 0; c < dim; ++c)
        gw[(size_t)i * dim + c] = W[i] > 0.0 ? a * gb[(size_t)i * dim + c] / W[i] : 0.0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t m = 0; m < n; ++m) {
      double acc_m[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (W[m] == 0.0)
        for (int32_t c = 0; c < dim; ++c) acc_m[c] = a * gb[(size_t)m * dim + c];
      for (int32_t j = 0; j < n; ++j) {
        if (j == m) continue;
        double d = D[(size_t)m * n + j];
        double w = w_of(d);
        if (w == 0.0) continue;
        const double* xm = X + (size_t)m * dim;
        const double* xj = X + (size_t)j * dim;
        double r = dist(dim, xm, xj);
        const double* gm = gw + (size_t)m * dim;
        const double* gj = gw + (size_t)j * dim;
        /* sum_j w_mj g_j */
        for (int32_t c = 0; c < dim; ++c) acc_m[c] += w * gj[c];
        if (r == 0.0) continue;
        /* P_mj (g_m - g_j) = (1/(d r)) [e - u (u . e)],  e = g_m - g_j */
        double ue = 0.0;
        for (int32_t c = 0; c < dim; ++c) ue += (xm[c] - xj[c]) / r * (gm[c] - gj[c]);
        for (int32_t c = 0; c < dim; ++c)
          acc_m[c] += ((gm[c] - gj[c]) - (xm[c] - xj[c]) / r * ue) / (d * r);
        /* row m's use of d_mj */
        double t = 0.0;
        for (int32_t c = 0; c < dim; ++c)
          t += gm[c] * (-2.0 * w / d * (xj[c] - XH[(size_t)m * dim + c]) - w * (xm[c] - xj[c]) / r);
        gD[(size_t)m * n + j] += t;
      }
      for (int32_t c = 0; c < dim; ++c) gn[(size_t)m * dim + c] = acc_m[c] - b * gb[(size_t)m * dim + c];
    }
    memcpy(gb, gn, sizeof(double) * nd);
  }
  memcpy(gX0, gb, sizeof(double) * nd);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t j = i + 1; j < n; ++j) {
      double s = gD[(size_t)i * n + j] + gD[(size_t)j * n + i];
      gD[(size_t)i * n + j] = s;
      gD[(size_t)j * n + i] = s;
    }
  free(Xs); free(XHs); free(W); free(gb); free(gw); free(gn);
  return SLO_OK;
}

/* dL/dlen for every CSR entry, by the chain rule through the shortest paths:
 * the distance of a pair s < t is the length of the tree path from s to t in
 * the tree of source s (pred, n x n), so every edge on that path receives
 * gD[s][t].  Both CSR entries of an edge get the edge's derivative.  Walks
 * every pair's path explicitly. */
int slo_edge_grad(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, const int32_t* P, const double* gD,
                  double* glen) {
  int64_t nnz = row_ptr[n];
  double* ge = (double*)calloc((size_t)(nnz > 0 ? nnz : 1), sizeof(double));
  if (!ge) return SLO_ENOMEM;
  for (int32_t s = 0; s < n; ++s) {
    const int32_t* pr = P + (size_t)s * n;
    for (int32_t t = s + 1; t < n; ++t) {
      if (pr[t] < 0) continue;
      double g = gD[(size_t)s * n + t];
      int32_t v = t;
      while (v != s) {
        int32_t u = pr[v];
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
          if (col_idx[e] == u) ge[e] += g;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
          if (col_idx[e] == v) ge[e] += g;
        v = u;
      }
    }
  }
  memcpy(glen, ge, sizeof(double) * (size_t)nnz);
  free(ge);
  return SLO_OK;
}

/* ====================================================================== */
/* Graph forms for layouts too large for an n x n distance matrix.         */
/* Each row's distances come from the graph (slo_sssp) when the row is     */
/* needed and are dropped after it, so memory is O(n) per thread.  Every   */
/* row is the same row function as the matrix form, and row sums are added */
/* in the same order, so the results equal the matrix forms bit for bit.   */
/* ====================================================================== */

/* X^H of the Jacobi step (eq. 5, one sweep from X) for every vertex. */
int slo_h_jacobi_graph(int32_t n, int32_t dim, const int64_t* row_ptr, const int32_t* col_idx, const double* len,
                       const double* X, double* XH) {
  int status = SLO_OK;
#pragma omp parallel
  {
    double* drow = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!drow) {
#pragma omp critical
      status = SLO_ENOMEM;
    }
#pragma omp for schedule(dynamic, 64)
    for (int32_t i = 0; i < n; ++i) {
      if (!drow) continue;
      int r = slo_sssp(n, row_ptr, col_idx, len, i, drow);
      if (r != SLO_OK) {
#pragma omp critical
        status = r;
        continue;
      }
      slo_h_jacobi_row(n, dim, drow, i, X, XH + (size_t)i * dim);
    }
    free(drow);
  }
  return status;
}

/* f(XA) - f(XB) and its term scale, as slo_stress_delta. */
int slo_stress_delta_graph(int32_t n, int32_t dim, const int64_t* row_ptr, const int32_t* col_idx, const double* len,
                           const double* XA, const double* XB, double* delta, double* scale) {
  double* pd = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double* ps = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  int status = SLO_OK;
  if (!pd || !ps) { free(pd); free(ps); return SLO_ENOMEM; }
#pragma omp parallel
  {
    double* drow = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!drow) {
#pragma omp critical
      status = SLO_ENOMEM;
    }
#pragma omp for schedule(dynamic, 64)
    for (int32_t i = 0; i < n; ++i) {
      if (!drow) continue;
      int r = slo_sssp(n, row_ptr, col_idx, len, i, drow);
      if (r != SLO_OK) {
#pragma omp critical
        status = r;
        continue;
      }
      stress_delta_row(n, dim, drow, i, XA, XB, pd + i, ps + i);
    }
    free(drow);
  }
  double a = 0.0, b = 0.0;
  for (int32_t i = 0; i < n; ++i) { a += pd[i]; b += ps[i]; }
  *delta = a;
  *scale = b;
  free(pd);
  free(ps);
  return status;
}

/* The bounds of slo_stress_delta_bounds with each distance row found from */
/* the graph when needed, and from the same rows the difference and scale of */
/* slo_stress_delta: out = {U, L, sum |c m|, sum kappa |e|^2, delta, scale}. */
int slo_stress_delta_bounds_graph(int32_t n, int32_t dim, const int64_t* row_ptr, const int32_t* col_idx,
                                  const double* len, const double* XA, const double* XB, double out[6]) {
  double* part = (double*)malloc(sizeof(double) * 6 * (size_t)(n > 0 ? n : 1));
  int status = SLO_OK;
  if (!part) return SLO_ENOMEM;
#pragma omp parallel
  {
    double* drow = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!drow) {
#pragma omp critical
      status = SLO_ENOMEM;
    }
#pragma omp for schedule(dynamic, 64)
    for (int32_t i = 0; i < n; ++i) {
      if (!drow) continue;
      int r = slo_sssp(n, row_ptr, col_idx, len, i, drow);
      if (r != SLO_OK) {
#pragma omp critical
        status = r;
        continue;
      }
      stress_bounds_row(n, dim, drow, i, XA, XB, part + 6 * (size_t)i);
      stress_delta_row(n, dim, drow, i, XA, XB, part + 6 * (size_t)i + 4, part + 6 * (size_t)i + 5);
    }
    free(drow);
  }
  double t[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int32_t i = 0; i < n; ++i)
    for (int k = 0; k < 6; ++k) t[k] += part[6 * (size_t)i + k];
  t[1] = t[0] - t[3];
  for (int k = 0; k < 6; ++k) out[k] = t[k];
  free(part);
  return status;
}

/* ====================================================================== */
/* Probabilistic strategy (Sec. 5.2): the paper's factor of each iteration */
/* is drawn by roulette from {0.5, 1.0, 1.5, 2.0} with probabilities       */
/* 0.3, 0.3, 0.2, 0.2.  The draw of iteration g (counted from the start of */
/* the layout, so a resumed run continues the sequence) uses the uniform   */
/* variate u = (z >> 11) * 2^-53, z = the output number g (from 0) of the   */
/* SplitMix64 generator seeded with `seed` (Steele, Lea and Flood, "Fast    */
/* splittable pseudorandom number generators", OOPSLA 2014):               */
/*   state_g = seed + (g + 1) * 0x9E3779B97F4A7C15 (mod 2^64), then the    */
/*   finalizer z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;         */
/*   z *= 0x94D049BB133111EB; z ^= z >> 31.                                 */
/* The roulette takes the first factor whose cumulative probability        */
/* exceeds u: u < 0.3 -> 0.5, u < 0.6 -> 1.0, u < 0.8 -> 1.5, else 2.0.     */
/* ====================================================================== */
uint64_t slo_splitmix64(uint64_t seed, uint64_t g) {
  uint64_t z = seed + (g + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* out[k] = the paper's factor of iteration first + k, k < count. */
void slo_auto_factors(uint64_t seed, int64_t first, int32_t count, double* out) {
  for (int32_t k = 0; k < count; ++k) {
    const double u = (double)(slo_splitmix64(seed, (uint64_t)(first + k)) >> 11) * 0x1.0p-53;
    out[k] = u < 0.3 ? 0.5 : u < 0.6 ? 1.0 : u < 0.8 ? 1.5 : 2.0;
  }
}
