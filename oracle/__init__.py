"""Oracle for the SOR-accelerated stress-majorization layout.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; never by the product package,
which shares no code with it.

A thin ctypes wrapper over ``sorlayout_oracle.c``: plain IEEE-double C that
writes out the paper's definitions (Wang & Wang 2012): the stress (eq. 1), the
Laplacians and majorant (Prop. 2.1, eq. 2), the majorization step as the
solution of eq. 5 (Prop. 2.3) in three orderings, and Algorithm 2 with the
extrapolation of eq. 10/11, and the reverse-mode derivative of the unrolled
iteration (initial placement and, through the shortest paths, edge lengths).
See the C file for the definitions; this module only marshals numpy arrays.

Relaxation factor convention: ``omega`` is the classical factor, the paper's
factor is ``omega - 1`` (``omega = 1`` is Algorithm 1).

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against hand-computed cases, closed forms, invariants and the convergence
theory of Sec. 3; see each test for its pin.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sorlayout_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

JACOBI, EXACT, GAUSS_SEIDEL = 0, 1, 2
_ORDERINGS = {"jacobi": JACOBI, "exact": EXACT, "gauss_seidel": GAUSS_SEIDEL, "gs": GAUSS_SEIDEL}
TRACE_COLS = 8


def build(force: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (IEEE double, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-std=c99", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Result(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rejected", ctypes.c_int32), ("status", ctypes.c_int32),
                ("residual", ctypes.c_double)]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            i32, f64 = ctypes.c_int32, ctypes.c_double
            sig = {
                "slo_sssp": (ctypes.c_int, [i32, P, P, P, i32, P]),
                "slo_apsp": (ctypes.c_int, [i32, P, P, P, P]),
                "slo_sssp_rows": (ctypes.c_int, [i32, P, P, P, P, i32, P]),
                "slo_weight_sums": (None, [i32, P, P]),
                "slo_stress": (f64, [i32, i32, P, P]),
                "slo_stress_delta": (None, [i32, i32, P, P, P, P, P]),
                "slo_stress_delta_bounds": (None, [i32, i32, P, P, P, P]),
                "slo_stress_delta_bounds_graph": (ctypes.c_int, [i32, i32, P, P, P, P, P, P]),
                "slo_apply_LW": (None, [i32, i32, P, P, P]),
                "slo_apply_LY": (None, [i32, i32, P, P, P]),
                "slo_majorant": (f64, [i32, i32, P, P, P]),
                "slo_h_jacobi": (None, [i32, i32, P, P, P]),
                "slo_h_jacobi_rows": (None, [i32, i32, P, P, i32, P, P]),
                "slo_h_gauss_seidel": (None, [i32, i32, P, P, P]),
                "slo_exact_prepare": (P, [i32, P]),
                "slo_exact_free": (None, [P]),
                "slo_h_exact": (ctypes.c_int, [P, i32, P, P, P]),
                "slo_residual": (f64, [i32, i32, P, P]),
                "slo_layout": (ctypes.c_int, [i32, i32, P, P, f64, f64, i32, i32, i32, i32, P, P, i32, P, P,
                                              ctypes.POINTER(_Result)]),
                "slo_sp_trees": (ctypes.c_int, [i32, P, P, P, P, P]),
                "slo_stress_grad": (None, [i32, i32, P, P, P]),
                "slo_layout_vjp": (ctypes.c_int, [i32, i32, P, P, f64, i32, P, P, P, P]),
                "slo_edge_grad": (ctypes.c_int, [i32, P, P, P, P, P]),
                "slo_h_jacobi_graph": (ctypes.c_int, [i32, i32, P, P, P, P, P]),
                "slo_stress_delta_graph": (ctypes.c_int, [i32, i32, P, P, P, P, P, P, P]),
                "slo_splitmix64": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_uint64]),
                "slo_auto_factors": (None, [ctypes.c_uint64, ctypes.c_int64, i32, P]),
            }
            for name, (res, args) in sig.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _csr(row_ptr, col_idx, lengths):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    ln = None if lengths is None else _f64(lengths)
    return rp, ci, ln


def _check(status, what):
    if status != 0:
        raise RuntimeError("oracle %s failed with status %d" % (what, status))


# --------------------------------------------------------------------------
# Ideal distances (shortest paths; Sec. 2 and 5.1)
# --------------------------------------------------------------------------
def apsp(row_ptr, col_idx, lengths=None) -> np.ndarray:
    """All-pairs shortest-path distances, n x n, +inf between components."""
    lib = _load()
    rp, ci, ln = _csr(row_ptr, col_idx, lengths)
    n = len(rp) - 1
    D = np.empty((n, n), dtype=np.float64)
    _check(lib.slo_apsp(n, _p(rp), _p(ci), _p(ln), _p(D)), "apsp")
    return D


def sssp_rows(row_ptr, col_idx, rows, lengths=None) -> np.ndarray:
    """Shortest-path distance rows for the given source vertices."""
    lib = _load()
    rp, ci, ln = _csr(row_ptr, col_idx, lengths)
    n = len(rp) - 1
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.empty((len(rows), n), dtype=np.float64)
    _check(lib.slo_sssp_rows(n, _p(rp), _p(ci), _p(ln), _p(rows), len(rows), _p(out)), "sssp_rows")
    return out


def weight_sums(D) -> np.ndarray:
    """W_i = sum_j d_ij^-2, the diagonal of L^W (Prop. 2.1)."""
    lib = _load()
    D = _f64(D)
    n = D.shape[0]
    W = np.empty(n, dtype=np.float64)
    lib.slo_weight_sums(n, _p(D), _p(W))
    return W


# --------------------------------------------------------------------------
# Stress and majorant (eq. 1, Prop. 2.1)
# --------------------------------------------------------------------------
def stress(D, X) -> float:
    lib = _load()
    D, X = _f64(D), _f64(X)
    return float(lib.slo_stress(D.shape[0], X.shape[1], _p(D), _p(X)))


def stress_delta(D, XA, XB):
    """(f(XA) - f(XB) summed pair by pair, sum of the absolute pair terms)."""
    lib = _load()
    D, XA, XB = _f64(D), _f64(XA), _f64(XB)
    a, b = ctypes.c_double(), ctypes.c_double()
    lib.slo_stress_delta(D.shape[0], XA.shape[1], _p(D), _p(XA), _p(XB), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def stress_delta_bounds(D, XA, XB):
    """(U, L, sum |c m|, sum kappa |e|^2): U >= f(XA) - f(XB) >= L from the
    pair terms' first-order parts (see the C source)."""
    lib = _load()
    D, XA, XB = _f64(D), _f64(XA), _f64(XB)
    out = np.zeros(4)
    lib.slo_stress_delta_bounds(D.shape[0], XA.shape[1], _p(D), _p(XA), _p(XB), _p(out))
    return tuple(float(v) for v in out)


def stress_delta_bounds_graph(row_ptr, col_idx, XA, XB, lengths=None):
    """stress_delta_bounds with each distance row found from the graph when
    needed, followed by stress_delta's (difference, scale) from the same rows:
    (U, L, sum |c m|, sum kappa |e|^2, f(XA) - f(XB), scale)."""
    lib = _load()
    rp, ci, ln = _csr(row_ptr, col_idx, lengths)
    XA, XB = _f64(XA), _f64(XB)
    out = np.zeros(6)
    _check(lib.slo_stress_delta_bounds_graph(XA.shape[0], XA.shape[1], _p(rp), _p(ci), _p(ln), _p(XA), _p(XB),
                                             _p(out)), "stress_delta_bounds_graph")
    return tuple(float(v) for v in out)


def stress_delta_graph(row_ptr, col_idx, XA, XB, lengths=None):
    """stress_delta with each distance row found from the graph when needed."""
    lib = _load()
    rp, ci, ln = _csr(row_ptr, col_idx, lengths)
    XA, XB = _f64(XA), _f64(XB)
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(lib.slo_stress_delta_graph(XA.shape[0], XA.shape[1], _p(rp), _p(ci), _p(ln), _p(XA), _p(XB),
                                      ctypes.byref(a), ctypes.byref(b)), "stress_delta_graph")
    return a.value, b.value


def apply_LW(D, X) -> np.ndarray:
    lib = _load()
    D, X = _f64(D), _f64(X)
    out = np.empty_like(X)
    lib.slo_apply_LW(D.shape[0], X.shape[1], _p(D), _p(X), _p(out))
    return out


def apply_LY(D, Y) -> np.ndarray:
    lib = _load()
    D, Y = _f64(D), _f64(Y)
    out = np.empty_like(Y)
    lib.slo_apply_LY(D.shape[0], Y.shape[1], _p(D), _p(Y), _p(out))
    return out


def majorant(D, X, Y) -> float:
    lib = _load()
    D, X, Y = _f64(D), _f64(X), _f64(Y)
    return float(lib.slo_majorant(D.shape[0], X.shape[1], _p(D), _p(X), _p(Y)))


# --------------------------------------------------------------------------
# Majorization step H (eq. 5) in three orderings
# --------------------------------------------------------------------------
def h_jacobi(D, X) -> np.ndarray:
    lib = _load()
    D, X = _f64(D), _f64(X)
    XH = np.empty_like(X)
    lib.slo_h_jacobi(D.shape[0], X.shape[1], _p(D), _p(X), _p(XH))
    return XH


def h_jacobi_rows(Drows, rows, X) -> np.ndarray:
    """x^H of the listed vertices; Drows[k] is the distance row of rows[k]."""
    lib = _load()
    Drows, X = _f64(Drows), _f64(X)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.empty((len(rows), X.shape[1]), dtype=np.float64)
    lib.slo_h_jacobi_rows(X.shape[0], X.shape[1], _p(Drows), _p(rows), len(rows), _p(X), _p(out))
    return out


def h_jacobi_graph(row_ptr, col_idx, X, lengths=None) -> np.ndarray:
    """X^H of the Jacobi step for every vertex, each distance row found from
    the graph when it is needed (no n x n matrix): equals h_jacobi(apsp(...), X)."""
    lib = _load()
    rp, ci, ln = _csr(row_ptr, col_idx, lengths)
    X = _f64(X)
    XH = np.empty_like(X)
    _check(lib.slo_h_jacobi_graph(X.shape[0], X.shape[1], _p(rp), _p(ci), _p(ln), _p(X), _p(XH)), "h_jacobi_graph")
    return XH


def h_gauss_seidel(D, X) -> np.ndarray:
    lib = _load()
    D, X = _f64(D), _f64(X)
    XH = np.empty_like(X)
    lib.slo_h_gauss_seidel(D.shape[0], X.shape[1], _p(D), _p(X), _p(XH))
    return XH


def h_exact(D, X) -> np.ndarray:
    lib = _load()
    D, X = _f64(D), _f64(X)
    ctx = lib.slo_exact_prepare(D.shape[0], _p(D))
    if not ctx:
        raise RuntimeError("oracle exact factorization failed")
    try:
        XH = np.empty_like(X)
        _check(lib.slo_h_exact(ctx, X.shape[1], _p(D), _p(X), _p(XH)), "h_exact")
    finally:
        lib.slo_exact_free(ctx)
    return XH


def residual(X, XH) -> float:
    lib = _load()
    X, XH = _f64(X), _f64(XH)
    return float(lib.slo_residual(X.shape[0], X.shape[1], _p(X), _p(XH)))


# --------------------------------------------------------------------------
# Algorithm 2 driver
# --------------------------------------------------------------------------
def layout(D, X0, omega=1.0, tol=1e-3, max_iter=200, ordering="jacobi", safeguard=True,
           trace_stress=False, trace_positions=False, omega_schedule=None, omega_vertex=None,
           enumerate=False):
    """Run Algorithm 2 (Algorithm 1 at omega = 1) from X0.

    Relaxation strategies (Sec. 5.2): a fixed ``omega``; ``omega_schedule``
    (one classical factor per iteration, e.g. drawn by the roulette of the
    probabilistic strategy); ``enumerate`` (argmin over the paper's candidates
    0, 0.5, ..., 9); ``omega_vertex`` (one classical factor per vertex).

    Returns ``(X, info)``; ``info`` holds iterations, converged, rejected,
    residual, the per-iteration ``trace`` (columns: residual, accepted,
    f(X~) - f(X^H), its term scale, f(X^k), paper's factor used, enumerating
    gap and its scale) and, when asked, ``positions`` (placement after every
    iteration).
    """
    lib = _load()
    D = _f64(D)
    X = _f64(X0).copy()
    n, dim = X.shape
    order = _ORDERINGS[ordering] if isinstance(ordering, str) else int(ordering)
    trace = np.full((max(max_iter, 1), TRACE_COLS), np.nan)
    xtrace = np.empty((max(max_iter, 1), n, dim)) if trace_positions else None
    res = _Result()
    sched = None if omega_schedule is None else _f64(omega_schedule)
    if sched is not None and len(sched) < max_iter:
        raise ValueError("omega_schedule needs max_iter entries")
    vert = None if omega_vertex is None else _f64(omega_vertex)
    if vert is not None and len(vert) != n:
        raise ValueError("omega_vertex needs n entries")
    st = lib.slo_layout(n, dim, _p(D), _p(X), float(omega), float(tol), int(max_iter), order,
                        int(bool(safeguard)), int(bool(trace_stress)), _p(sched), _p(vert), int(bool(enumerate)),
                        _p(trace), _p(xtrace), ctypes.byref(res))
    _check(st, "layout")
    k = res.iterations
    info = {"iterations": k, "converged": bool(res.converged), "rejected": res.rejected,
            "residual": res.residual, "trace": trace[:k].copy()}
    if trace_positions:
        info["positions"] = xtrace[:k].copy()
    return X, info


# Probabilistic strategy (Sec. 5.2): roulette over the paper's factors
# 0.5, 1.0, 1.5, 2.0 with probabilities 0.3, 0.3, 0.2, 0.2.
AUTO_FACTORS = (0.5, 1.0, 1.5, 2.0)
AUTO_PROBS = (0.3, 0.3, 0.2, 0.2)


def splitmix64(seed: int, g: int) -> int:
    """Output number g (from 0) of SplitMix64 seeded with seed."""
    return int(_load().slo_splitmix64(int(seed) & (2 ** 64 - 1), int(g)))


def auto_factors(seed: int, first: int, count: int) -> np.ndarray:
    """The paper's factors the probabilistic strategy draws at iterations
    first .. first + count - 1 (SplitMix64 variate of the iteration index)."""
    out = np.empty(max(int(count), 0), dtype=np.float64)
    _load().slo_auto_factors(int(seed) & (2 ** 64 - 1), int(first), int(count), _p(out))
    return out


ENUM_FACTORS = tuple(0.5 * c for c in range(19))


# --------------------------------------------------------------------------
# Derivatives of the unrolled iteration (reverse mode, FP64)
# --------------------------------------------------------------------------
def sp_trees(row_ptr, col_idx, lengths):
    """(D, pred): shortest-path distances for positive edge lengths and the
    shortest-path tree of every source (pred[s][v] = lowest-numbered neighbour
    on a shortest path, -1 for s and unreachable v).  D is made symmetric from
    its upper triangle: d_ts := d_st for s < t (the tree of the lower-numbered
    end defines the pair)."""
    lib = _load()
    rp, ci, ln = _csr(row_ptr, col_idx, lengths)
    n = len(rp) - 1
    D = np.empty((n, n), dtype=np.float64)
    P = np.empty((n, n), dtype=np.int32)
    _check(lib.slo_sp_trees(n, _p(rp), _p(ci), _p(ln), _p(D), _p(P)), "sp_trees")
    iu = np.triu_indices(n, 1)
    D.T[iu] = D[iu]
    return D, P


def stress_grad(D, X) -> np.ndarray:
    """Gradient of eq. 1 with respect to X."""
    lib = _load()
    D, X = _f64(D), _f64(X)
    G = np.empty_like(X)
    lib.slo_stress_grad(D.shape[0], X.shape[1], _p(D), _p(X), _p(G))
    return G


def layout_vjp(D, X0, omega, iters, accepted, G):
    """(dL/dX0, dL/dD) for L a function of X^K after K = iters Jacobi-SOR
    iterations with the safeguard decisions held at ``accepted`` (trace column
    1 of ``layout``); G = dL/dX^K.  dL/dD is symmetric: d_ij and d_ji are one
    variable."""
    lib = _load()
    D, X0, G = _f64(D), _f64(X0), _f64(G)
    acc = _f64(accepted)
    n, dim = X0.shape
    assert len(acc) >= iters
    gX0 = np.empty_like(X0)
    gD = np.empty((n, n), dtype=np.float64)
    _check(lib.slo_layout_vjp(n, dim, _p(D), _p(X0), float(omega), int(iters), _p(acc), _p(G), _p(gX0), _p(gD)),
           "layout_vjp")
    return gX0, gD


def edge_grad(row_ptr, col_idx, pred, gD) -> np.ndarray:
    """dL/dlen per CSR entry from dL/dD through the shortest-path trees."""
    lib = _load()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    P = np.ascontiguousarray(pred, dtype=np.int32)
    gD = _f64(gD)
    n = len(rp) - 1
    out = np.empty(int(rp[-1]), dtype=np.float64)
    _check(lib.slo_edge_grad(n, _p(rp), _p(ci), _p(P), _p(gD), _p(out)), "edge_grad")
    return out
