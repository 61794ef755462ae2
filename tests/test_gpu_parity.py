"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (FP32 device arithmetic against an FP64 reference):
  * distances and every integer result: bit-exact
  * W_i (FP64 on both sides, same summation order): rtol 1e-12
  * one Jacobi step X^H: max_i ||x_i^gpu - x_i^orc|| <= 1e-5 * diam(X^k)
    (each pair term carries ~1e-7 relative error and the forces are summed in
    FP64 per 16-pair group; diam = bounding-box diagonal)
  * free run: max_i ||x_i^gpu(k) - x_i^orc(k)|| <= 1e-4 * diam(X^orc(k)) for
    every iteration k; safeguard decisions equal unless the oracle's
    f(X~) - f(X^H) lies within 64 * 2^-24 of the sum of its absolute pair
    terms, in which case the comparison of that run ends at that iteration
  * iterations to tol: equal, or +-1 when the oracle's residual at its
    stopping iteration lies within 0.1% of tol; final stress: rtol 1e-4
"""
import os

import numpy as np
import pytest

import oracle
from fixtures import GOLDEN, ppi_fig4a
from lockstep import check_safeguard_lockstep
from paper_1711_01228_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

AMBIG = 64 * 2.0 ** -24


@pytest.fixture(scope="module")
def sl():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    from paper_1711_01228_amd import binding

    return binding


def diam(X):
    return float(np.linalg.norm(X.max(0) - X.min(0)))


def oracle_D(g):
    return oracle.apsp(g.row_ptr, g.col_idx)


def as_u8(D):
    out = np.where(np.isfinite(D), D, 0.0)
    assert out.max() <= 255
    return out.astype(np.uint8)


def dev(X):
    return torch.tensor(np.asarray(X, dtype=np.float32), device="cuda").contiguous()


def ppi_graph():
    n, edges, _ = ppi_fig4a()
    return inputs.to_csr(n, edges, name="ppi")


def small_graphs():
    return {
        "grid16": inputs.grid16(0)[0],
        "ppi": ppi_graph(),
        "er300_sparse": inputs.erdos_renyi(300, 280, 7),
        "tree500": inputs.random_tree(500, 3),
        "ba2000": inputs.barabasi_albert(2000, 3, 11),
        "ragged_129": inputs.erdos_renyi(129, 400, 5),
        # a hub of degree 219 (14 chunks of the BFS gather), its leaves and a path
        "star260": inputs.to_csr(260, [(0, k) for k in range(1, 220)] + [(k, k + 1) for k in range(220, 259)] +
                                 [(5, 220)]),
        "k40": inputs.complete_graph(40),  # every row longer than one gather run
    }


# ---------------------------------------------------------------------------
# distances and weights (plan creation)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", sorted(small_graphs()))
def test_distances_and_weights(sl, name):
    g = small_graphs()[name]
    print("case", name, g.n, flush=True)
    D = oracle_D(g)
    with sl.Plan(g, 2) as plan:
        got = plan.distance_rows(np.arange(g.n))
        np.testing.assert_array_equal(got, as_u8(D))
        np.testing.assert_allclose(plan.weights(), oracle.weight_sums(D), rtol=1e-12, atol=0)


SWEEP = 8192  # sources of one breadth-first sweep of the library


def multi_sweep_graphs():
    """Graphs searched in several sweeps of SWEEP sources."""
    # a star of SWEEP vertices with two paths of 100 hung on its centre: the
    # first sweep (the star) is 101 levels deep, the second (the paths) 200, so
    # the second outlasts the levels queued from the first sweep's depth
    S = SWEEP
    edges = [(0, k) for k in range(1, S)] + [(0, S), (0, S + 100)]
    edges += [(k, k + 1) for k in range(S, S + 99)] + [(k, k + 1) for k in range(S + 100, S + 199)]
    return {
        "two_tails_%d" % (S + 200): inputs.to_csr(S + 200, edges),
        "er9000_components": inputs.erdos_renyi(9000, 7000, 9),  # isolated vertices and many components
    }


@pytest.mark.parametrize("name", sorted(multi_sweep_graphs()))
def test_distances_and_weights_several_sweeps(sl, name):
    g = multi_sweep_graphs()[name]
    print("case", name, g.n, flush=True)
    D = oracle_D(g)
    with sl.Plan(g, 2) as plan:
        np.testing.assert_array_equal(plan.distance_rows(np.arange(g.n)), as_u8(D))
        np.testing.assert_allclose(plan.weights(), oracle.weight_sums(D), rtol=1e-12, atol=0)


def test_distances_er4096_and_ba65536_sampled(sl):
    for g in (inputs.er4096(0)[0], inputs.ba65536(2)[0]):
        print("case", g.name, flush=True)
        rows = np.unique(np.concatenate([np.arange(0, g.n, max(1, g.n // 61)), [g.n - 1, 1, 63, 64, 65]]))
        D = oracle.sssp_rows(g.row_ptr, g.col_idx, rows)
        with sl.Plan(g, 2) as plan:
            np.testing.assert_array_equal(plan.distance_rows(rows), as_u8(D))
            W = plan.weights()
        w = np.where((D > 0) & np.isfinite(D), 1.0 / np.where(D > 0, D, 1.0) ** 2, 0.0).sum(1)
        np.testing.assert_allclose(W[rows], w, rtol=1e-12)


def test_distances_four_sweeps_and_a_deeper_last_sweep(sl):
    """Four sweeps queued after the first one's depth: the last sweep (two paths
    of 7 hung on the star's centre and on a leaf) is 15 levels deep where the
    first is 9, so it is redone after the others.  Sampled rows bit-exact
    against the oracle's BFS, W to rounding."""
    S = SWEEP
    n_leaves = 3 * S - 1
    edges = [(0, k) for k in range(1, n_leaves + 1)]
    p0 = n_leaves + 1                       # path P from the centre
    edges += [(0, p0)] + [(p0 + k, p0 + k + 1) for k in range(6)]
    q0 = p0 + 7                             # path Q from leaf 1
    edges += [(1, q0)] + [(q0 + k, q0 + k + 1) for k in range(6)]
    n = q0 + 7
    g = inputs.to_csr(n, edges)
    print("case star_two_paths", n, flush=True)
    rows = np.unique(np.concatenate([np.arange(0, n, 997), [0, 1, 2, S, 2 * S, 3 * S - 1, p0, p0 + 6, q0, q0 + 6,
                                                            n - 1]]))
    D = oracle.sssp_rows(g.row_ptr, g.col_idx, rows)
    assert D[np.searchsorted(rows, p0 + 6)].max() == 15 and D[np.searchsorted(rows, 2)].max() == 9
    with sl.Plan(g, 2) as plan:
        np.testing.assert_array_equal(plan.distance_rows(rows), as_u8(D))
        W = plan.weights()
    w = np.where((D > 0) & np.isfinite(D), 1.0 / np.where(D > 0, D, 1.0) ** 2, 0.0).sum(1)
    np.testing.assert_allclose(W[rows], w, rtol=1e-12)


def test_distance_above_255_hops_is_refused(sl):
    g = inputs.path_graph(300)
    with pytest.raises(sl.SlError) as e:
        sl.Plan(g, 2)
    assert e.value.status == sl.SL_ERANGE
    with sl.Plan(inputs.path_graph(256), 2) as plan:  # longest distance 255: fits
        assert plan.distance_rows([0])[0, 255] == 255


# ---------------------------------------------------------------------------
# one step and stress
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("name", sorted(small_graphs()))
def test_one_jacobi_step(sl, name, dim):
    g = small_graphs()[name]
    print("case", name, dim, flush=True)
    X0 = inputs.uniform_positions(g.n, dim, seed=77, lo=0.0, hi=float(np.sqrt(g.n)))
    D = oracle_D(g)
    XH = oracle.h_jacobi(D, X0)
    X = dev(X0)
    with sl.Plan(g, dim) as plan:
        info = plan.run(X, omega=1.0, tol=0.0, max_iter=1)
        assert info["iterations"] == 1
        err = np.abs(X.cpu().numpy().astype(np.float64) - XH).max()
        assert err <= 1e-5 * diam(X0), err
        f_gpu = plan.stress(dev(X0))
    assert f_gpu == pytest.approx(oracle.stress(D, X0), rel=1e-5)


# ---------------------------------------------------------------------------
# free runs against the oracle trajectory
# ---------------------------------------------------------------------------
def compare_runs(g, X0, D, omega, iters, safeguard=True, sl=None, dim=2, **kw):
    Xo, io = oracle.layout(D, X0, omega=omega, tol=0.0, max_iter=iters, safeguard=safeguard,
                           trace_positions=True)
    X = dev(X0)
    with sl.Plan(g, dim) as plan:
        ig = plan.run(X, omega=omega, tol=0.0, max_iter=iters, safeguard=safeguard, trace=True,
                      trace_positions=True, **kw)
    assert ig["iterations"] == iters == io["iterations"]
    Pg, Po = ig["positions"].astype(np.float64), io["positions"]
    tg, to = ig["trace"], io["trace"]
    compared = 0
    for k in range(iters):
        if tg[k, 1] != to[k, 1]:
            # a flipped safeguard decision is only acceptable inside the rounding band
            assert abs(to[k, 2]) <= AMBIG * to[k, 3], (k, to[k], tg[k])
            break
        err = np.abs(Pg[k] - Po[k]).max()
        assert err <= 1e-4 * diam(Po[k]), (k, err, diam(Po[k]))
        # residual: FP32 storage of x^H bounds its accuracy to ~1e-7 absolute
        np.testing.assert_allclose(tg[k, 0], to[k, 0], rtol=2e-3, atol=2e-6)
        compared += 1
    if safeguard:  # every iteration, from the GPU's own iterate
        check_safeguard_lockstep(D, X0, ig)
    return compared, ig, io


FORCE_PASSES = {"default": {}, "unordered": {"sym_force": True}}


@pytest.mark.parametrize("force", sorted(FORCE_PASSES))
@pytest.mark.parametrize("omega", [1.0, 1.5])
def test_grid16_free_run_200_iterations(sl, omega, force):
    g, X0 = inputs.grid16(0)
    print("case grid16 omega", omega, force, flush=True)
    compared, ig, io = compare_runs(g, X0, oracle_D(g), omega, 200, sl=sl, **FORCE_PASSES[force])
    assert compared >= 150
    if omega == 1.0:
        assert np.all(ig["trace"][:, 1] == -1)


@pytest.mark.parametrize("force", sorted(FORCE_PASSES))
@pytest.mark.parametrize("dim", [2, 3])
def test_ppi_free_run_with_rejections(sl, dim, force):
    g = ppi_graph()
    X0 = inputs.uniform_positions(g.n, dim, seed=5)
    print("case ppi omega 3.0 dim", dim, force, flush=True)
    compared, ig, io = compare_runs(g, X0, oracle_D(g), 3.0, 60, sl=sl, dim=dim, **FORCE_PASSES[force])
    assert compared >= 30
    assert io["rejected"] > 0  # a long stride is refused at least once


def test_no_safeguard_free_run(sl):
    g = small_graphs()["ragged_129"]
    X0 = inputs.uniform_positions(g.n, 2, seed=9, hi=10.0)
    compared, ig, io = compare_runs(g, X0, oracle_D(g), 1.3, 40, safeguard=False, sl=sl)
    assert compared == 40 and ig["rejected"] == 0


def _read_sweep():
    rows = {}
    with open(os.path.join(GOLDEN, "er4096_sweep.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            om, it, conv, rej, res_last, res_prev, fin = line.split()
            rows[float(om)] = dict(iterations=int(it), converged=int(conv), rejected=int(rej),
                                   res_last=float(res_last), res_prev=float(res_prev), stress=float(fin))
    return rows


@pytest.mark.parametrize("omega", [1.0, 1.2, 1.4, 1.6])
def test_er4096_iterations_to_tol(sl, omega):
    ref = _read_sweep()[omega]
    g, X0 = inputs.er4096(0)
    print("case er4096 omega", omega, flush=True)
    X = dev(X0)
    with sl.Plan(g, 2) as plan:
        info = plan.run(X, omega=omega, tol=1e-3, max_iter=2000)
    assert info["converged"] == ref["converged"]
    near = abs(ref["res_last"] - 1e-3) <= 1e-6 or abs(ref["res_prev"] - 1e-3) <= 1e-6
    assert abs(info["iterations"] - ref["iterations"]) <= (1 if near else 0), (info, ref)
    assert info["stress"] == pytest.approx(ref["stress"], rel=1e-4)


@pytest.mark.parametrize("force", sorted(FORCE_PASSES))
@pytest.mark.parametrize("omega", [1.0, 1.6])
def test_er4096_first_iterations_track_oracle(sl, omega, force):
    g, X0 = inputs.er4096(0)
    print("case er4096 omega", omega, force, flush=True)
    compared, _, _ = compare_runs(g, X0, oracle_D(g), omega, 25, sl=sl, **FORCE_PASSES[force])
    assert compared >= 20


def test_rel_stress_drop_is_the_last_iterations_relative_decrease(sl):
    g, X0 = inputs.grid16(5)
    D = oracle_D(g)
    for omega, iters in ((1.0, 7), (1.5, 12)):
        X = dev(X0)
        with sl.Plan(g, 2) as plan:
            info = plan.run(X, omega=omega, tol=0.0, max_iter=iters, trace=True, trace_positions=True)
            none = plan.run(dev(X0), omega=omega, tol=0.0, max_iter=iters, final_stress=False)
            zero = plan.run(dev(X0), omega=omega, max_iter=0)
        P = info["positions"].astype(np.float64)
        f_prev, f_last = oracle.stress(D, P[-2]), oracle.stress(D, P[-1])
        assert info["stress"] == pytest.approx(f_last, rel=1e-5)
        assert info["rel_stress_drop"] == pytest.approx((f_prev - f_last) / f_prev, rel=1e-4, abs=1e-6)
        assert np.isnan(none["rel_stress_drop"]) and np.isnan(zero["rel_stress_drop"])


# ---------------------------------------------------------------------------
# full size: BA n = 65536, sampled rows of one step in the benchmark's launch shape
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_ba65536_one_step_sampled_rows(sl, dim):
    g, X0 = inputs.ba65536(dim)
    print("case ba65536 dim", dim, flush=True)
    rng = np.random.default_rng(dim)
    rows = np.unique(np.concatenate([rng.choice(g.n, 60, replace=False), [0, 1, 63, 64, g.n - 1]]))
    Drows = oracle.sssp_rows(g.row_ptr, g.col_idx, rows)
    XH_rows = oracle.h_jacobi_rows(Drows, rows, X0)
    X = dev(X0)
    with sl.Plan(g, dim) as plan:
        np.testing.assert_array_equal(plan.distance_rows(rows), as_u8(Drows))
        info = plan.run(X, omega=1.0, tol=0.0, max_iter=1)
    assert info["iterations"] == 1
    got = X.cpu().numpy().astype(np.float64)[rows]
    err = np.abs(got - XH_rows).max()
    assert err <= 1e-5 * diam(X0), err


@pytest.mark.parametrize("dim", [2, 3])
def test_ba_above_full_size_ragged_sampled_rows(sl, dim):
    """A graph larger than the benchmark's, of a ragged size: BA n = 100,003,
    m = 3 (n_pad = 100,032, so the last row block and column group are partial;
    13 sweeps of the search, the last with 1,699 sources; 10 GB of distance
    bytes), in 2-D and 3-D.  Sampled distance rows bit-exact against the oracle's
    BFS, their W to rounding, and the rows of one Jacobi step within the FP32 bound."""
    g, X0 = inputs.ba65536(dim, n=100003)
    print("case ba100003 dim", dim, flush=True)
    rng = np.random.default_rng(11)
    edge = [0, 1, 63, 64, 8191, 8192, 98303, 98304, 99999, g.n - 1]
    rows = np.unique(np.concatenate([rng.choice(g.n, 60, replace=False), edge]))
    Drows = oracle.sssp_rows(g.row_ptr, g.col_idx, rows)
    XH_rows = oracle.h_jacobi_rows(Drows, rows, X0)
    X = dev(X0)
    with sl.Plan(g, dim) as plan:
        np.testing.assert_array_equal(plan.distance_rows(rows), as_u8(Drows))
        W = plan.weights()
        info = plan.run(X, omega=1.0, tol=0.0, max_iter=1)
    w = np.where((Drows > 0) & np.isfinite(Drows), 1.0 / np.where(Drows > 0, Drows, 1.0) ** 2, 0.0).sum(1)
    np.testing.assert_allclose(W[rows], w, rtol=1e-12)
    assert info["iterations"] == 1
    got = X.cpu().numpy().astype(np.float64)[rows]
    err = np.abs(got - XH_rows).max()
    assert err <= 1e-5 * diam(X0), err


# (dimension, iteration k from 0): both take the fused pass over unordered pairs
# (the bounds of the safeguard, the exact difference when they leave its sign
# open); each case costs the oracle two passes over all pairs with every distance
# row found by breadth-first search (~25 s on 16 threads)
BA_LOCKSTEP = [(2, 0), (2, 1), (2, 2), (3, 1)]


@pytest.mark.parametrize("dim,k", BA_LOCKSTEP)
def test_ba65536_safeguard_lockstep(sl, dim, k):
    """The launch configuration the benchmark times (n = 65,536, omega = 1.5,
    the safeguard summed inside the pass that takes the next force at X~).
    Iteration k from the GPU's own X^k: the oracle forms X^H for every vertex,
    X~ and f(X~) - f(X^H) (distance rows found from the graph one at a time,
    never the n x n matrix), and these are compared with the GPU's trace
    column 2 (within 1e-4 of the value or the FP32 band 64 * 2^-24 of the term
    scale), its decision (equal outside that band) and all rows of X^{k+1}
    (X~ or X^H by the oracle's decision, within 1e-5 of the layout's
    diameter)."""
    g, X0 = inputs.ba65536(dim)
    omega = 1.5
    print("case ba65536 lockstep dim", dim, "iteration", k, flush=True)
    X = dev(X0)
    with sl.Plan(g, dim) as plan:
        info = plan.run(X, omega=omega, tol=0.0, max_iter=k + 1, trace=True, trace_positions=True,
                        final_stress=False)
    assert info["iterations"] == k + 1
    P = info["positions"].astype(np.float64)
    Xk = X0 if k == 0 else P[k - 1]
    XH = oracle.h_jacobi_graph(g.row_ptr, g.col_idx, Xk)
    XT = XH + (omega - 1.0) * (XH - Xk)
    tg = info["trace"][k]
    if np.isfinite(tg[5]):  # the unordered pass reports the bounds U >= f(X~) - f(X^H) >= L
        u, lo, su, q, df, scale = oracle.stress_delta_bounds_graph(g.row_ptr, g.col_idx, XT, XH)
        print("bounds: U gpu %.10g oracle %.10g, L gpu %.10g oracle %.10g (scales %.4g, %.4g)"
              % (tg[5], u, tg[6], lo, su, q), flush=True)
        assert abs(tg[5] - u) <= max(1e-4 * abs(u), AMBIG * (su + q))
        if np.isfinite(tg[6]):
            assert abs(tg[6] - lo) <= max(1e-4 * abs(lo), AMBIG * (su + q))
        assert lo <= df <= u
    else:
        df, scale = oracle.stress_delta_graph(g.row_ptr, g.col_idx, XT, XH)
    print("f(X~) - f(X^H): gpu %.10g oracle %.10g scale %.4g; decision gpu %g" % (tg[2], df, scale, tg[1]),
          flush=True)
    if np.isnan(tg[2]):  # decided by a bound
        assert (tg[5] <= 0.0) if tg[1] == 1.0 else (tg[6] > 0.0)
    else:
        assert abs(tg[2] - df) <= max(1e-4 * abs(df), AMBIG * scale)
    take = df <= 0.0
    if abs(df) > AMBIG * scale:
        assert tg[1] == (1.0 if take else 0.0)
    else:  # inside the FP32 band either decision is correct: follow the GPU's
        take = tg[1] == 1.0
    expect = XT if take else XH
    err = np.abs(P[k] - expect).max()
    assert err <= 1e-5 * max(diam(Xk), diam(XH)), err


# ---------------------------------------------------------------------------
# edge cases and run-to-run behaviour
# ---------------------------------------------------------------------------
def test_degenerate_graphs(sl):
    # n = 1: nothing to do; converged with no step
    g1 = inputs.to_csr(1, [])
    X = dev([[0.25, 0.5]])
    with sl.Plan(g1, 2) as plan:
        info = plan.run(X, omega=1.5, max_iter=10)
    assert info["iterations"] == 0 and info["converged"] == 1
    np.testing.assert_array_equal(X.cpu().numpy(), [[0.25, 0.5]])
    # two vertices, one edge: the Jacobi step oscillates between r = 1.5 and 0.5
    g2 = inputs.to_csr(2, [(0, 1)])
    X = dev([[0.0, 0.0], [0.5, 0.0]])
    with sl.Plan(g2, 2) as plan:
        info = plan.run(X, omega=1.0, tol=1e-6, max_iter=3)
    assert info["iterations"] == 3 and info["converged"] == 0
    # hand value (tests/golden/hand_cases.txt); rsq/rcp round to ~1 ulp
    np.testing.assert_allclose(X.cpu().numpy(), [[-0.5, 0.0], [1.0, 0.0]], rtol=0, atol=1e-6)
    # isolated vertices keep their place; max_iter = 0 leaves X alone
    g = inputs.to_csr(6, [(0, 1), (1, 2)])
    X0 = inputs.uniform_positions(6, 2, 3)
    X = dev(X0)
    with sl.Plan(g, 2) as plan:
        plan.run(X, omega=1.5, tol=0.0, max_iter=5)
        np.testing.assert_array_equal(X.cpu().numpy()[3:], X0[3:].astype(np.float32))
        X2 = dev(X0)
        info = plan.run(X2, max_iter=0)
        assert info["iterations"] == 0
        np.testing.assert_array_equal(X2.cpu().numpy(), X0.astype(np.float32))
    # no edges at all: one step, nothing moves, converged
    g0 = inputs.to_csr(5, [])
    X = dev(inputs.uniform_positions(5, 3, 1))
    with sl.Plan(g0, 3) as plan:
        info = plan.run(X, max_iter=4)
    assert info["iterations"] == 1 and info["converged"] == 1


def test_non_finite_start_is_reported(sl):
    g = inputs.grid_graph(4, 4)
    X0 = inputs.uniform_positions(16, 2, 1)
    X0[5, 0] = np.nan
    X = dev(X0)
    with sl.Plan(g, 2) as plan:
        with pytest.raises(sl.SlError) as e:
            plan.run(X, max_iter=3)
    assert e.value.status == sl.SL_ENUMERIC


def test_bitwise_repeatable_graph_and_resume(sl):
    g, X0 = inputs.grid16(1)
    with sl.Plan(g, 2) as plan:
        outs = []
        for use_graph, chunk in ((True, 0), (True, 7), (False, 0)):
            X = dev(X0)
            plan.run(X, omega=1.5, tol=0.0, max_iter=40, use_graph=use_graph, check_every=chunk)
            outs.append(X.cpu().numpy())
        X = dev(X0)
        plan.run(X, omega=1.5, tol=0.0, max_iter=20)
        plan.run(X, omega=1.5, tol=0.0, max_iter=20)  # resume from iterate 20
        outs.append(X.cpu().numpy())
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])


def test_no_final_stress_keeps_the_iterates(sl):
    g, X0 = inputs.grid16(1)
    with sl.Plan(g, 2) as plan:
        Xa, Xb = dev(X0), dev(X0)
        ra = plan.run(Xa, omega=1.5, tol=1e-3, max_iter=300)
        rb = plan.run(Xb, omega=1.5, tol=1e-3, max_iter=300, final_stress=False)
        assert np.isnan(rb["stress"]) and np.isfinite(ra["stress"])
        assert (ra["iterations"], ra["rejected"], ra["residual"]) == (rb["iterations"], rb["rejected"], rb["residual"])
        np.testing.assert_array_equal(Xa.cpu().numpy(), Xb.cpu().numpy())
        assert plan.stress(Xb) == ra["stress"]  # the same pass, asked for separately


def test_layout_one_call_matches_plan(sl):
    g, X0 = inputs.grid16(2)
    X1, info = sl.layout(g, X0, omega=1.5, tol=1e-3, max_iter=500)
    X = dev(X0)
    with sl.Plan(g, 2) as plan:
        info2 = plan.run(X, omega=1.5, tol=1e-3, max_iter=500)
    np.testing.assert_array_equal(X1.cpu().numpy(), X.cpu().numpy())
    assert info["iterations"] == info2["iterations"] and info["converged"]
    assert info["plan_ms"] > 0 and info["run_ms"] > 0


def test_probe_rates_are_plausible(sl):
    import bench

    # lane operations per second: 1,024 SIMDs x 16 lanes x ~2.4 GHz is ~3.9e13 at one instruction per 4 cycles
    for kind in ("fma", "rsq", "sqrt", "rcp"):
        per_s, ms = bench.probe_rate(kind)
        print(kind, per_s, ms, flush=True)
        assert ms > 0.0 and 1e12 < per_s < 1.6e14
