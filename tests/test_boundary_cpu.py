"""Host-side checks of the C-ABI library and the input generators (no GPU).

The library loads without a GPU; validation runs before any HIP call, so
every malformed-input path is exercised here.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1711_01228_amd import binding as b
from paper_1711_01228_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sorlayout.h")
PROBE_HEADER = os.path.join(ROOT, "include", "slprobe.h")


def declared_functions(header=HEADER, prefix="sl_"):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(%s[a-z0-9_]+)\s*\(" % prefix, text)))


def exported_symbols(path):
    out = subprocess.run(["nm", "-D", "--defined-only", path], stdout=subprocess.PIPE, text=True).stdout
    return set(re.findall(r"\sT\s+(\S+)", out))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(b.LIB, name), name
    exported = exported_symbols(b.LIB_PATH)
    assert set(names) <= exported
    assert set(b.EXPORTED) == set(names)
    # the calibration probe is the benchmark's own library, not part of the method's ABI
    assert not any(name.startswith("slp_") or "probe" in name for name in exported)


def test_probe_library_exports_its_header():
    from paper_1711_01228_amd import build_lib

    names = declared_functions(PROBE_HEADER, "slp_")
    assert names == ["slp_probe_rate"]
    assert set(names) <= exported_symbols(build_lib.PROBE_LIB)


def test_default_options():
    o = b.sl_options()
    b.LIB.sl_default_options(ctypes.byref(o))
    assert (o.dim, o.max_iter, o.omega, o.tol, o.safeguard, o.flags) == (2, 1000, 1.0, 1e-3, 1, 0)
    assert b.LIB.sl_validate(None, ctypes.byref(o)) == b.SL_EINVAL  # graph is required


class G:
    def __init__(self, n, row_ptr, col_idx, edge_len=None):
        self.n, self.row_ptr, self.col_idx, self.edge_len = n, np.asarray(row_ptr), np.asarray(col_idx), edge_len


def _tri():
    g = inputs.grid_graph(2, 2)
    return G(g.n, g.row_ptr.copy(), g.col_idx.copy())


@pytest.mark.parametrize("mutate,msg", [
    (lambda g: setattr(g, "n", -1), "negative"),
    (lambda g: g.row_ptr.__setitem__(0, 1), "row_ptr[0]"),
    (lambda g: g.row_ptr.__setitem__(2, 1), "decreases"),
    (lambda g: g.col_idx.__setitem__(0, 7), "outside"),
    (lambda g: g.col_idx.__setitem__(0, 0), "self loop"),
    (lambda g: g.col_idx.__setitem__(1, g.col_idx[0]), "duplicate"),
])
def test_validation_rejects_malformed_graphs(mutate, msg):
    g = _tri()
    mutate(g)
    if g.n < 0:
        ga = b._GraphArgs(0, g.row_ptr, g.col_idx)
        ga.s.n = -1
        st = b.LIB.sl_validate(ctypes.byref(ga.s), None)
    else:
        st = b.sl_validate_status(g)
    assert st == b.SL_EINVAL
    assert msg in b.last_error()


def test_validation_rejects_asymmetric_and_nnz_mismatch():
    # 0 -> 1 without 1 -> 0
    g = G(2, [0, 1, 1], [1])
    assert b.sl_validate_status(g) == b.SL_EINVAL and "symmetric" in b.last_error()
    ga = b.graph_args(_tri())
    ga.s.nnz = ga.s.nnz + 1
    assert b.LIB.sl_validate(ctypes.byref(ga.s), None) == b.SL_EINVAL and "nnz" in b.last_error()


def test_edge_length_validation():
    g = _tri()
    g.edge_len = np.ones(len(g.col_idx), dtype=np.float32)
    assert b.sl_validate_status(g) == b.SL_OK
    g.edge_len[2] = -1.0
    assert b.sl_validate_status(g) == b.SL_EINVAL and "positive" in b.last_error()
    g.edge_len[2] = np.nan
    assert b.sl_validate_status(g) == b.SL_EINVAL
    g.edge_len[2] = 2.0  # its twin entry still holds 1.0
    assert b.sl_validate_status(g) == b.SL_EINVAL and "two different lengths" in b.last_error()
    big = inputs.path_graph(b.SL_WEIGHTED_MAX_N + 1)
    big.edge_len = np.ones(big.nnz, dtype=np.float32)
    assert b.sl_validate_status(big) == b.SL_ENOTSUP


@pytest.mark.parametrize("field,value", [
    ("dim", 1), ("dim", 4), ("omega", 0.0), ("omega", float("nan")), ("omega", float("inf")),
    ("omega", 17.0), ("tol", -1e-3), ("tol", float("nan")), ("max_iter", -1), ("safeguard", 2), ("flags", 64),
    ("iter_offset", -1), ("strategy", 4), ("seed", 5),  # a seed without the probabilistic strategy
])
def test_validation_rejects_bad_options(field, value):
    o = b.make_options()
    setattr(o, field, value)
    assert b.sl_validate_status(_tri(), o) == b.SL_EINVAL
    assert b.last_error()


def test_probabilistic_strategy_and_resume_options():
    b.sl_validate(_tri(), b.make_options(strategy=b.SL_OMEGA_AUTO, seed=2 ** 64 - 1, iter_offset=10 ** 6))
    # a schedule is read at the global iterations iter_offset .. iter_offset + max_iter - 1
    sched = np.array([0.0, 0.0, 1.5, 2.0, 2.5])
    b.sl_validate(_tri(), b.make_options(strategy=b.SL_OMEGA_SCHEDULE, omega_schedule=sched, max_iter=3,
                                         iter_offset=2))
    o = b.make_options(strategy=b.SL_OMEGA_SCHEDULE, omega_schedule=sched, max_iter=3, iter_offset=1)
    assert b.sl_validate_status(_tri(), o) == b.SL_EINVAL and "omega_schedule[1]" in b.last_error()


def test_result_and_options_layout_match_the_header():
    # the new fields sit at the end of each struct, after the ones of the first layout
    assert b.sl_options.seed.offset == b.sl_options.reserved3.offset + 4
    assert b.sl_options.iter_offset.offset == b.sl_options.seed.offset + 8
    assert ctypes.sizeof(b.sl_options) == b.sl_options.iter_offset.offset + 8
    assert b.sl_result.rel_stress_drop.offset == b.sl_result.run_ms.offset + 8


def test_valid_inputs_and_empty_graph():
    b.sl_validate(_tri(), b.make_options(dim=3, omega=2.5, tol=0.0, max_iter=0, safeguard=False))
    b.sl_validate(_tri(), b.make_options(final_stress=False, ordered_force=True, separate_safeguard=True))
    b.sl_validate(G(0, [0], []))
    b.sl_validate(G(3, [0, 0, 0, 0], []))  # isolated vertices only


def test_plan_create_rejects_before_device_work():
    # validation fails before any HIP call, so this runs without a GPU
    g = _tri()
    g.col_idx[0] = 0
    with pytest.raises(b.SlError) as e:
        b.sl_plan_create(g, 2, stream=0)
    assert e.value.status == b.SL_EINVAL
    with pytest.raises(b.SlError) as e:
        b.sl_plan_create(_tri(), 5, stream=0)
    assert e.value.status == b.SL_EINVAL


# ---------------------------------------------------------------------------
# input generators
# ---------------------------------------------------------------------------
def _is_connected(g):
    seen = np.zeros(g.n, bool)
    stack = [0]
    seen[0] = True
    while stack:
        u = stack.pop()
        for v in g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]]:
            if not seen[v]:
                seen[v] = True
                stack.append(v)
    return seen.all()


def test_generators_shapes_and_validity():
    g = inputs.grid_graph(16, 16)
    assert (g.n, g.num_edges) == (256, 480)
    er = inputs.erdos_renyi(4096, 12288, seed=2000)
    assert (er.n, er.num_edges) == (4096, 12288)
    ba = inputs.barabasi_albert(2000, 3, seed=3000)
    assert ba.num_edges == 6 + 3 * (2000 - 4) and _is_connected(ba)
    t = inputs.random_tree(500, seed=1)
    assert t.num_edges == 499 and _is_connected(t)
    for gg in (g, er, ba, t):
        b.sl_validate(gg)
    # deterministic in the seed
    np.testing.assert_array_equal(inputs.erdos_renyi(300, 500, 9).col_idx, inputs.erdos_renyi(300, 500, 9).col_idx)
    X = inputs.uniform_positions(1000, 3, seed=4, lo=0.0, hi=64.0)
    assert X.min() >= 0 and X.max() < 64
    np.testing.assert_array_equal(X, X.astype(np.float32).astype(np.float64))


def test_ba_degree_is_heavy_tailed():
    ba = inputs.barabasi_albert(20000, 3, seed=5)
    deg = np.diff(ba.row_ptr)
    assert deg.min() >= 3 and deg.max() > 100


def test_probe_rate_refuses_unknown_kind_before_any_device_call():
    import bench

    lib = bench.probe_library()
    per_s, ms = ctypes.c_double(0.0), ctypes.c_double(0.0)
    assert lib.slp_probe_rate(4, None, ctypes.byref(per_s), ctypes.byref(ms)) == -1
    assert lib.slp_probe_rate(0, None, None, ctypes.byref(ms)) == -1



# ---------------------------------------------------------------------------
# allocation-free batched layout: everything it refuses, it refuses before any
# device work (so without a GPU)
# ---------------------------------------------------------------------------
def _noalloc_status(gs, dim=2, batch=None):
    args = batch if batch is not None else b.BatchArgs(gs)
    opt = b.make_options(dim, 1.5, 1e-3, 10, True)
    tot = b.sl_result()
    return b.LIB.sl_batch_layout_noalloc(ctypes.byref(args.s), None, ctypes.byref(opt), None, None,
                                         ctypes.byref(tot))


def test_noalloc_refuses_a_batch_beyond_its_scratch():
    # 17 distance blocks of 1 MiB (n_pad 1024) exceed the 16 MiB array
    assert _noalloc_status([inputs.grid_graph(32, 32)] * 17) == b.SL_EINVAL
    msg = b.last_error()
    assert "SL_NOALLOC_SCRATCH_BYTES" in msg and str(16 * 1024 * 1024) in msg
    # too many graphs for the host staging, whatever their size
    assert _noalloc_status([inputs.to_csr(1, [])] * 4097) == b.SL_EINVAL and "graphs" in b.last_error()


def test_noalloc_validates_like_the_plan():
    args = b.BatchArgs([inputs.path_graph(4)])
    args.graph_ptr = np.array([0, 2, 4], dtype=np.int64)
    args.s.num_graphs, args.s.graph_ptr = 2, args.graph_ptr.ctypes.data
    assert _noalloc_status(None, batch=args) == b.SL_EINVAL and "leaves graph" in b.last_error()
    assert _noalloc_status([inputs.grid_graph(33, 32)]) == b.SL_EINVAL and "more than 1024" in b.last_error()
    # a duplicate entry, then an asymmetric one
    g = inputs.to_csr(3, [(0, 1), (1, 2)])
    dup = inputs.Graph(3, np.array([0, 2, 4, 5], dtype=np.int64), np.array([1, 1, 0, 2, 1], dtype=np.int32),
                       name="dup")
    assert _noalloc_status([g, dup]) == b.SL_EINVAL and "duplicate" in b.last_error()
    asym = inputs.to_csr(3, [(0, 1)])
    asym.col_idx = np.array([1, 2], dtype=np.int32)  # row 0 -> 1, row 1 -> 2: no reverse entries
    asym.row_ptr = np.array([0, 1, 2, 2], dtype=np.int64)
    assert _noalloc_status([asym]) == b.SL_EINVAL and "not symmetric" in b.last_error()
    # after those errors the validation bitmap is clean: a valid batch gets as
    # far as the option check (dim 4 is refused after the batch checks)
    assert _noalloc_status([g, inputs.grid_graph(4, 4)], dim=4) == b.SL_EINVAL and "dim" in b.last_error()


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU: asked for more (or started as one rank of
    several) it exits with a message before any device work."""
    for args, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})):
        r = subprocess.run(["python3", os.path.join(ROOT, "bench.py")] + args, capture_output=True, text=True,
                           timeout=120, env=dict(os.environ, **env))
        assert r.returncode != 0 and r.stdout == ""
        assert "one GPU only" in r.stderr
