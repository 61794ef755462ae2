"""ctypes binding of libsorlayout (include/sorlayout.h).

Argument marshalling only: every step of the layout runs in the HIP library.
Device buffers and streams come from PyTorch (``tensor.data_ptr()``,
``torch.cuda.current_stream().cuda_stream``); torch does no arithmetic here.
Importing this module fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsorlayout.so")

SL_OK, SL_EINVAL, SL_ENOMEM, SL_EDEVICE, SL_ERANGE, SL_ENUMERIC, SL_ENOTSUP = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "SL_OK", -1: "SL_EINVAL", -2: "SL_ENOMEM", -3: "SL_EDEVICE", -4: "SL_ERANGE",
                -5: "SL_ENUMERIC", -6: "SL_ENOTSUP"}
SL_TRACE_COLS = 7
SL_FLAG_TRACE_STRESS = 1
SL_FLAG_NO_GRAPH = 2
SL_FLAG_SYM_FORCE = 4
SL_FLAG_SEPARATE_SAFEGUARD = 8
SL_FLAG_ORDERED_FORCE = 16
SL_FLAG_NO_FINAL_STRESS = 32
SL_OMEGA_FIXED, SL_OMEGA_SCHEDULE, SL_OMEGA_ENUM, SL_OMEGA_AUTO = 0, 1, 2, 3
STRATEGIES = {"fixed": SL_OMEGA_FIXED, "schedule": SL_OMEGA_SCHEDULE, "enum": SL_OMEGA_ENUM, "auto": SL_OMEGA_AUTO}
SL_ORDER_JACOBI, SL_ORDER_EXACT = 0, 1
ORDERINGS = {"jacobi": SL_ORDER_JACOBI, "exact": SL_ORDER_EXACT}

EXPORTED = ("sl_default_options", "sl_validate", "sl_plan_create", "sl_plan_run", "sl_plan_stress",
            "sl_plan_distance_rows", "sl_plan_weights", "sl_plan_profile", "sl_plan_destroy", "sl_layout",
            "sl_last_error", "sl_batch_plan_create", "sl_batch_plan_tune", "sl_batch_plan_run",
            "sl_batch_plan_destroy", "sl_plan_distance_rows_f32", "sl_plan_tree_rows", "sl_plan_set_lengths",
            "sl_plan_stress_grad", "sl_plan_unroll", "sl_plan_unroll_backward", "sl_batch_layout_noalloc")
SL_WEIGHTED_MAX_N = 16384
SL_BATCH_MAX_N = 1024
SL_BATCH_CLASSES = 16


class SlError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


class sl_graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("edge_len", ctypes.c_void_p)]


class sl_options(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("omega", ctypes.c_double),
                ("tol", ctypes.c_double), ("safeguard", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("ordering", ctypes.c_int32), ("trace", ctypes.c_void_p),
                ("xtrace", ctypes.c_void_p), ("strategy", ctypes.c_int32), ("reserved2", ctypes.c_int32),
                ("omega_schedule", ctypes.c_void_p), ("omega_vertex", ctypes.c_void_p),
                ("inner_tol", ctypes.c_double), ("inner_max_iter", ctypes.c_int32), ("reserved3", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("iter_offset", ctypes.c_int64)]


class sl_batch(ctypes.Structure):
    _fields_ = [("num_graphs", ctypes.c_int32), ("graph_ptr", ctypes.c_void_p), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


class sl_result(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("rejected", ctypes.c_int32),
                ("inner_iterations", ctypes.c_int32), ("residual", ctypes.c_double), ("stress", ctypes.c_double),
                ("plan_ms", ctypes.c_double), ("run_ms", ctypes.c_double), ("rel_stress_drop", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    # PyTorch ships its own HIP runtime under the same soname (libamdhip64.so.7)
    # as the one the library links.  Whichever is loaded first serves the whole
    # process, so torch is imported first: one runtime for torch's allocations
    # and streams and for the library's kernels.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsorlayout.so is not built (%s); run __graft_entry__.build() or "
                          "python -m paper_1711_01228_amd.build_lib" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int
    sigs = {
        "sl_default_options": (None, [ctypes.POINTER(sl_options)]),
        "sl_validate": (st, [ctypes.POINTER(sl_graph), ctypes.POINTER(sl_options)]),
        "sl_plan_create": (st, [ctypes.POINTER(sl_graph), i32, P, ctypes.POINTER(P)]),
        "sl_plan_run": (st, [P, P, ctypes.POINTER(sl_options), P, ctypes.POINTER(sl_result)]),
        "sl_plan_stress": (st, [P, P, i32, P, ctypes.POINTER(ctypes.c_double)]),
        "sl_plan_distance_rows": (st, [P, P, i32, P, P]),
        "sl_plan_weights": (st, [P, P, P]),
        "sl_plan_distance_rows_f32": (st, [P, P, i32, P, P]),
        "sl_plan_tree_rows": (st, [P, P, i32, P, P]),
        "sl_plan_set_lengths": (st, [P, P, P]),
        "sl_plan_stress_grad": (st, [P, P, i32, P, ctypes.POINTER(ctypes.c_double), P]),
        "sl_plan_unroll": (st, [P, P, ctypes.POINTER(sl_options), i32, P, ctypes.POINTER(sl_result)]),
        "sl_plan_unroll_backward": (st, [P, P, P, P, P]),
        "sl_plan_profile": (st, [P, P, i32, ctypes.c_double, i32, P, P]),
        "sl_plan_destroy": (st, [P]),
        "sl_layout": (st, [ctypes.POINTER(sl_graph), P, ctypes.POINTER(sl_options), P, ctypes.POINTER(sl_result)]),
        "sl_last_error": (ctypes.c_char_p, []),
        "sl_batch_plan_create": (st, [ctypes.POINTER(sl_batch), i32, P, ctypes.POINTER(P)]),
        "sl_batch_plan_tune": (st, [P, P, ctypes.POINTER(sl_options), P, P]),
        "sl_batch_plan_run": (st, [P, P, ctypes.POINTER(sl_options), P, P, ctypes.POINTER(sl_result)]),
        "sl_batch_plan_destroy": (st, [P]),
        "sl_batch_layout_noalloc": (st, [ctypes.POINTER(sl_batch), P, ctypes.POINTER(sl_options), P, P,
                                         ctypes.POINTER(sl_result)]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = _load()


def last_error() -> str:
    return LIB.sl_last_error().decode()


def _check(status):
    if status != SL_OK:
        raise SlError(status, last_error())


class _GraphArgs:
    """Keeps the CSR arrays alive for the duration of a call."""

    def __init__(self, n, row_ptr, col_idx, edge_len=None):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        self.edge_len = None if edge_len is None else np.ascontiguousarray(edge_len, dtype=np.float32)
        self.s = sl_graph(int(n), int(self.row_ptr[-1]) if len(self.row_ptr) else 0,
                          self.row_ptr.ctypes.data if len(self.row_ptr) else None,
                          self.col_idx.ctypes.data if len(self.col_idx) else None,
                          None if self.edge_len is None else self.edge_len.ctypes.data)


def graph_args(g) -> _GraphArgs:
    """From an object with n, row_ptr, col_idx (and optional edge_len)."""
    return _GraphArgs(g.n, g.row_ptr, g.col_idx, getattr(g, "edge_len", None))


def make_options(dim=2, omega=1.0, tol=1e-3, max_iter=1000, safeguard=True, check_every=0,
                 trace_stress=False, use_graph=True, trace=None, xtrace=None, strategy=SL_OMEGA_FIXED,
                 omega_schedule=None, omega_vertex=None, ordering=SL_ORDER_JACOBI, inner_tol=0.0,
                 inner_max_iter=0, sym_force=False, separate_safeguard=False, ordered_force=False,
                 final_stress=True, seed=0, iter_offset=0) -> sl_options:
    """omega_schedule: host float64 array (kept alive by the caller), indexed by
    the global iteration (iter_offset + k); omega_vertex: device pointer (int) or None."""
    o = sl_options()
    LIB.sl_default_options(ctypes.byref(o))
    o.dim, o.omega, o.tol, o.max_iter = int(dim), float(omega), float(tol), int(max_iter)
    o.safeguard, o.check_every = int(bool(safeguard)), int(check_every)
    o.flags = (SL_FLAG_TRACE_STRESS if trace_stress else 0) | (0 if use_graph else SL_FLAG_NO_GRAPH) | \
        (SL_FLAG_SYM_FORCE if sym_force else 0) | \
        (SL_FLAG_SEPARATE_SAFEGUARD if separate_safeguard else 0) | (SL_FLAG_ORDERED_FORCE if ordered_force else 0) | \
        (0 if final_stress else SL_FLAG_NO_FINAL_STRESS)
    o.trace = None if trace is None else int(trace)
    o.xtrace = None if xtrace is None else int(xtrace)
    o.strategy = int(strategy)
    o.omega_schedule = None if omega_schedule is None else omega_schedule.ctypes.data
    o.omega_vertex = None if omega_vertex is None else int(omega_vertex)
    o.ordering = int(ordering)
    o.inner_tol, o.inner_max_iter = float(inner_tol), int(inner_max_iter)
    o.seed, o.iter_offset = int(seed) & (2 ** 64 - 1), int(iter_offset)
    return o


def _stream_handle(stream):
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    return int(stream)


# --------------------------------------------------------------------------
# C-ABI entry points, same names
# --------------------------------------------------------------------------
def sl_validate(g, opt: sl_options | None = None) -> None:
    ga = graph_args(g)
    _check(LIB.sl_validate(ctypes.byref(ga.s), None if opt is None else ctypes.byref(opt)))


def sl_validate_status(g, opt: sl_options | None = None) -> int:
    ga = graph_args(g)
    return LIB.sl_validate(ctypes.byref(ga.s), None if opt is None else ctypes.byref(opt))


def sl_plan_create(g, dim: int, stream=None) -> int:
    ga = graph_args(g)
    h = ctypes.c_void_p()
    _check(LIB.sl_plan_create(ctypes.byref(ga.s), int(dim), _stream_handle(stream), ctypes.byref(h)))
    return h.value


def sl_plan_run(plan: int, X_ptr: int, opt: sl_options, stream=None) -> dict:
    res = sl_result()
    _check(LIB.sl_plan_run(plan, X_ptr, ctypes.byref(opt), _stream_handle(stream), ctypes.byref(res)))
    return res.as_dict()


def sl_plan_stress(plan: int, X_ptr: int, dim: int, stream=None) -> float:
    f = ctypes.c_double()
    _check(LIB.sl_plan_stress(plan, X_ptr, int(dim), _stream_handle(stream), ctypes.byref(f)))
    return f.value


def sl_plan_distance_rows(plan: int, rows, n: int, stream=None) -> np.ndarray:
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.zeros((len(rows), n), dtype=np.uint8)
    _check(LIB.sl_plan_distance_rows(plan, rows.ctypes.data, len(rows), _stream_handle(stream), out.ctypes.data))
    return out


def sl_plan_distance_rows_f32(plan: int, rows, n: int, stream=None) -> np.ndarray:
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.zeros((len(rows), n), dtype=np.float32)
    _check(LIB.sl_plan_distance_rows_f32(plan, rows.ctypes.data, len(rows), _stream_handle(stream), out.ctypes.data))
    return out


def sl_plan_tree_rows(plan: int, rows, n: int, stream=None) -> np.ndarray:
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.zeros((len(rows), n), dtype=np.int32)
    _check(LIB.sl_plan_tree_rows(plan, rows.ctypes.data, len(rows), _stream_handle(stream), out.ctypes.data))
    return out


def sl_plan_set_lengths(plan: int, edge_len, stream=None) -> None:
    ln = np.ascontiguousarray(edge_len, dtype=np.float32)
    _check(LIB.sl_plan_set_lengths(plan, ln.ctypes.data, _stream_handle(stream)))


def sl_plan_stress_grad(plan: int, X_ptr: int, dim: int, G_ptr: int, stream=None) -> float:
    f = ctypes.c_double()
    _check(LIB.sl_plan_stress_grad(plan, X_ptr, int(dim), _stream_handle(stream), ctypes.byref(f), G_ptr))
    return f.value


def sl_plan_unroll(plan: int, X_ptr: int, opt: sl_options, ckpt_every: int, stream=None) -> dict:
    res = sl_result()
    _check(LIB.sl_plan_unroll(plan, X_ptr, ctypes.byref(opt), int(ckpt_every), _stream_handle(stream),
                              ctypes.byref(res)))
    return res.as_dict()


def sl_plan_unroll_backward(plan: int, G_ptr: int, gX0_ptr: int, glen_ptr=None, stream=None) -> None:
    _check(LIB.sl_plan_unroll_backward(plan, G_ptr, gX0_ptr, glen_ptr, _stream_handle(stream)))


def sl_plan_weights(plan: int, n: int, stream=None) -> np.ndarray:
    W = np.zeros(n, dtype=np.float64)
    _check(LIB.sl_plan_weights(plan, _stream_handle(stream), W.ctypes.data))
    return W


def sl_plan_profile(plan: int, X_ptr: int, dim: int, omega: float, reps: int, stream=None) -> np.ndarray:
    ms = np.zeros(9, dtype=np.float64)
    _check(LIB.sl_plan_profile(plan, X_ptr, int(dim), float(omega), int(reps), _stream_handle(stream),
                               ms.ctypes.data))
    return ms


def sl_plan_destroy(plan: int) -> None:
    _check(LIB.sl_plan_destroy(plan))


def sl_layout(g, X_ptr: int, opt: sl_options, stream=None) -> dict:
    ga = graph_args(g)
    res = sl_result()
    _check(LIB.sl_layout(ctypes.byref(ga.s), X_ptr, ctypes.byref(opt), _stream_handle(stream), ctypes.byref(res)))
    return res.as_dict()


# --------------------------------------------------------------------------
# Convenience wrapper over torch tensors
# --------------------------------------------------------------------------
class Plan:
    """A plan on the current device: distances and weights of one graph."""

    def __init__(self, g, dim=2, stream=None):
        self.n, self.dim = int(g.n), int(dim)
        self.handle = sl_plan_create(g, dim, stream)

    def run(self, X, omega=1.0, tol=1e-3, max_iter=1000, safeguard=True, check_every=0, trace=False,
            trace_stress=False, trace_positions=False, use_graph=True, stream=None, strategy="fixed",
            omega_schedule=None, omega_vertex=None, ordering="jacobi", inner_tol=0.0, inner_max_iter=0,
            sym_force=False, separate_safeguard=False, ordered_force=False, final_stress=True, seed=0,
            iter_offset=0):
        """Run Algorithm 2 in place on the device tensor X (n x dim, float32).

        strategy: "fixed" (omega), "schedule" (omega_schedule, one classical
        factor per global iteration), "auto" (the probabilistic strategy of
        Sec. 5.2, drawn in the library from seed and the iteration number) or
        "enum" (argmin over the paper's factors 0, 0.5, ..., 9); omega_vertex:
        optional device tensor of n classical factors (fixed strategy).
        iter_offset: global number of the first iteration, for resuming a run
        (schedules and draws continue; trace rows stay local).  ordering: "jacobi" (one
        sweep of eq. 5) or "exact" (eq. 5 solved by conjugate gradients to
        inner_tol, at most inner_max_iter steps; 0 selects the defaults).
        sym_force / ordered_force: evaluate the force pass once per unordered
        pair (SL_FLAG_SYM_FORCE; Jacobi ordering; the default in 2-D from
        n_pad = 32768, 16384 for edge lengths) or over every ordered pair
        (SL_FLAG_ORDERED_FORCE).
        separate_safeguard: evaluate the safeguard in its own pass instead of
        inside the next force pass (SL_FLAG_SEPARATE_SAFEGUARD).
        final_stress=False skips the pass that evaluates f of the result
        (SL_FLAG_NO_FINAL_STRESS; ``stress`` is then NaN).
        Returns the sl_result fields; with ``trace`` also a ``trace`` array
        (iterations x 5) and with ``trace_positions`` the ``positions``
        (iterations x n x dim) on the host."""
        import torch

        if X.dtype != torch.float32 or not X.is_cuda or not X.is_contiguous() or tuple(X.shape) != (self.n, self.dim):
            raise ValueError("X must be a contiguous cuda float32 tensor of shape (%d, %d)" % (self.n, self.dim))
        tr = xt = None
        if trace or trace_stress:
            tr = torch.full((max(max_iter, 1), SL_TRACE_COLS), float("nan"), dtype=torch.float64, device=X.device)
        if trace_positions:
            xt = torch.zeros((max(max_iter, 1), self.n, self.dim), dtype=torch.float32, device=X.device)
        strat = STRATEGIES[strategy]
        sched = None if omega_schedule is None else np.ascontiguousarray(omega_schedule, dtype=np.float64)
        if sched is not None and len(sched) < iter_offset + max_iter:
            raise ValueError("omega_schedule needs iter_offset + max_iter entries")
        wv = None
        if omega_vertex is not None:
            wv = omega_vertex.to(device=X.device, dtype=torch.float32).contiguous()
        opt = make_options(self.dim, omega, tol, max_iter, safeguard, check_every, trace_stress, use_graph,
                           None if tr is None else tr.data_ptr(), None if xt is None else xt.data_ptr(),
                           strat, sched, None if wv is None else wv.data_ptr(), ORDERINGS[ordering], inner_tol,
                           inner_max_iter, sym_force, separate_safeguard, ordered_force, final_stress, seed,
                           iter_offset)
        info = sl_plan_run(self.handle, X.data_ptr(), opt, stream)
        k = info["iterations"]
        if tr is not None:
            info["trace"] = tr[:k].cpu().numpy()
        if xt is not None:
            info["positions"] = xt[:k].cpu().numpy()
        return info

    def stress(self, X, stream=None) -> float:
        return sl_plan_stress(self.handle, X.data_ptr(), self.dim, stream)

    def distance_rows(self, rows, stream=None) -> np.ndarray:
        return sl_plan_distance_rows(self.handle, rows, self.n, stream)

    def weights(self, stream=None) -> np.ndarray:
        return sl_plan_weights(self.handle, self.n, stream)

    def distance_rows_f32(self, rows, stream=None) -> np.ndarray:
        return sl_plan_distance_rows_f32(self.handle, rows, self.n, stream)

    def tree_rows(self, rows, stream=None) -> np.ndarray:
        return sl_plan_tree_rows(self.handle, rows, self.n, stream)

    def set_lengths(self, edge_len, stream=None) -> None:
        """New lengths per CSR entry (same graph); rebuilds distances and trees."""
        sl_plan_set_lengths(self.handle, edge_len, stream)

    def stress_grad(self, X, G, stream=None) -> float:
        """f(X) (eq. 1) and its gradient into the device tensor G (n x dim)."""
        return sl_plan_stress_grad(self.handle, X.data_ptr(), self.dim, G.data_ptr(), stream)

    def unroll(self, X, omega=1.5, iters=100, ckpt_every=10, safeguard=True, sym_force=False, ordered_force=False,
               stream=None) -> dict:
        """Exactly `iters` iterations in place on X, keeping the tape for
        unroll_backward; sym_force / ordered_force pick the force pass of the
        forward and the backward (default: the library's choice by size)."""
        opt = make_options(self.dim, omega, 0.0, iters, safeguard, sym_force=sym_force, ordered_force=ordered_force)
        return sl_plan_unroll(self.handle, X.data_ptr(), opt, ckpt_every, stream)

    def unroll_backward(self, G, gX0, glen=None, stream=None) -> None:
        """dL/dX0 (and dL/dlen per CSR entry) from G = dL/dX^K; device tensors."""
        sl_plan_unroll_backward(self.handle, G.data_ptr(), gX0.data_ptr(),
                                None if glen is None else glen.data_ptr(), stream)

    def profile(self, X, omega=1.5, reps=5, stream=None) -> dict:
        """Average device ms of each kernel of one iteration (HIP events)."""
        ms = sl_plan_profile(self.handle, X.data_ptr(), self.dim, omega, reps, stream)
        return dict(zip(("force", "update", "safeguard", "select", "lw_matvec", "force_sym",
                         "force_safeguard", "force_safeguard_sym", "force_safeguard_sym_exact"), ms.tolist()))

    def close(self):
        if self.handle:
            sl_plan_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def layout(g, X0, omega=1.0, tol=1e-3, max_iter=1000, **kw):
    """layout(G, X0, omega, tol, max_iter) -> (X, info) on the GPU.  X0 is a
    host array or a device tensor (n x dim); X is a new cuda float32 tensor."""
    import torch

    X = torch.as_tensor(np.asarray(X0, dtype=np.float32) if not torch.is_tensor(X0) else X0)
    X = X.to(device="cuda", dtype=torch.float32).contiguous().clone()
    with Plan(g, X.shape[1]) as plan:
        info = plan.run(X, omega=omega, tol=tol, max_iter=max_iter, **kw)
    return X, info


# --------------------------------------------------------------------------
# Batched layouts
# --------------------------------------------------------------------------
class BatchArgs:
    """Concatenation of many graphs into one block-diagonal CSR (global ids)."""

    def __init__(self, graphs):
        ns = np.fromiter((int(g.n) for g in graphs), dtype=np.int64, count=len(graphs))
        self.graph_ptr = np.zeros(len(graphs) + 1, dtype=np.int64)
        self.graph_ptr[1:] = np.cumsum(ns)
        rps = [np.asarray(g.row_ptr, dtype=np.int64) for g in graphs]
        nnz = np.fromiter((int(r[-1]) for r in rps), dtype=np.int64, count=len(graphs))
        e_ptr = np.zeros(len(graphs) + 1, dtype=np.int64)
        e_ptr[1:] = np.cumsum(nnz)
        self.row_ptr = np.zeros(int(self.graph_ptr[-1]) + 1, dtype=np.int64)
        if len(graphs):
            # each graph's row_ptr[1:] shifted by the entries before it
            np.concatenate([r[1:] for r in rps], out=self.row_ptr[1:])
            self.row_ptr[1:] += np.repeat(e_ptr[:-1], ns)
        if self.graph_ptr[-1] > np.iinfo(np.int32).max:
            raise ValueError("more than 2^31 - 1 vertices in the batch")
        # each graph's column indices shifted by the vertices before it (int32 ids)
        self.col_idx = np.zeros(int(e_ptr[-1]), dtype=np.int32)
        if int(e_ptr[-1]):
            np.concatenate([np.asarray(g.col_idx, dtype=np.int32) for g in graphs], out=self.col_idx)
            self.col_idx += np.repeat(self.graph_ptr[:-1].astype(np.int32), nnz)
        self.n_total = int(self.graph_ptr[-1])
        self.s = sl_batch(len(graphs), self.graph_ptr.ctypes.data, int(self.row_ptr[-1]), self.row_ptr.ctypes.data,
                          self.col_idx.ctypes.data if len(self.col_idx) else None)


def sl_batch_plan_create(batch: BatchArgs, dim: int, stream=None) -> int:
    h = ctypes.c_void_p()
    _check(LIB.sl_batch_plan_create(ctypes.byref(batch.s), int(dim), _stream_handle(stream), ctypes.byref(h)))
    return h.value


def sl_batch_plan_tune(plan: int, X_ptr: int, opt: sl_options, stream=None) -> np.ndarray:
    cfg = np.zeros(1 + SL_BATCH_CLASSES, dtype=np.int32)
    _check(LIB.sl_batch_plan_tune(plan, X_ptr, ctypes.byref(opt), _stream_handle(stream), cfg.ctypes.data))
    return cfg


def sl_batch_plan_run(plan: int, X_ptr: int, opt: sl_options, num_graphs: int, stream=None):
    per = (sl_result * max(num_graphs, 1))()
    tot = sl_result()
    _check(LIB.sl_batch_plan_run(plan, X_ptr, ctypes.byref(opt), _stream_handle(stream), per, ctypes.byref(tot)))
    return tot.as_dict(), [per[k].as_dict() for k in range(num_graphs)]


def sl_batch_plan_destroy(plan: int) -> None:
    _check(LIB.sl_batch_plan_destroy(plan))


def sl_batch_layout_noalloc(batch: BatchArgs, X_ptr: int, opt: sl_options, stream=None):
    """The allocation-free batched layout; returns (total, per-graph list)."""
    per = (sl_result * max(batch.s.num_graphs, 1))()
    tot = sl_result()
    _check(LIB.sl_batch_layout_noalloc(ctypes.byref(batch.s), X_ptr, ctypes.byref(opt), _stream_handle(stream), per,
                                       ctypes.byref(tot)))
    return tot.as_dict(), [per[k].as_dict() for k in range(batch.s.num_graphs)]


class BatchPlan:
    """Distances and weights of many small graphs (each n <= 1024) on the device."""

    def __init__(self, graphs, dim=2, stream=None):
        self.args = BatchArgs(graphs)
        self.num_graphs, self.dim = len(graphs), int(dim)
        self.graph_ptr = self.args.graph_ptr
        self.handle = sl_batch_plan_create(self.args, dim, stream)

    def _check_x(self, X):
        import torch

        if X.dtype != torch.float32 or not X.is_cuda or not X.is_contiguous() or \
                tuple(X.shape) != (self.args.n_total, self.dim):
            raise ValueError("X must be a contiguous cuda float32 tensor of shape (%d, %d)" % (self.args.n_total,
                                                                                          self.dim))

    def tune(self, X, omega=1.5, max_iter=8, safeguard=True, stream=None, tol=0.0) -> np.ndarray:
        """Autotune the launch; with tol > 0 the workgroup size is timed on whole runs to tol."""
        self._check_x(X)
        opt = make_options(self.dim, omega, tol, max_iter, safeguard)
        return sl_batch_plan_tune(self.handle, X.data_ptr(), opt, stream)

    def run(self, X, omega=1.5, tol=1e-3, max_iter=1000, safeguard=True, stream=None):
        """Lay out every graph in place; returns (total, per-graph list)."""
        self._check_x(X)
        opt = make_options(self.dim, omega, tol, max_iter, safeguard)
        return sl_batch_plan_run(self.handle, X.data_ptr(), opt, self.num_graphs, stream)

    def close(self):
        if self.handle:
            sl_batch_plan_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

