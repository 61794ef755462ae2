"""Pins of the oracle's derivatives (reverse mode through the unrolled
Jacobi-SOR iteration and the shortest paths), each against the definition of
the derivative or an invariance of the method:

  * central finite differences of the oracle's own forward run (FP64) for
    the initial placement, a single symmetric distance and an edge length
    (re-solving the shortest paths), with the safeguard decisions checked to
    stay the same under the perturbation;
  * translation and rotation invariance: sum_i dL/dx0_i = 0 and zero torque;
  * the weighted shortest-path trees against scipy's Dijkstra.
The loss is the stress (eq. 1) against hop distances at X^K.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import oracle
from paper_1711_01228_amd import inputs


def _weighted(n=40, m=90, seed=3):
    g = inputs.largest_component(inputs.erdos_renyi(n, m, seed))
    rng = np.random.default_rng(seed)
    e = g.edges()
    lens = 1.0 + rng.uniform(-0.1, 0.1, len(e))
    gw = inputs.to_csr(g.n, e, lens)
    return gw, gw.edge_len.astype(np.float64)


def _loss(Dhop, X):
    return oracle.stress(Dhop, X)


def _fd(fun, h=1e-5):
    """Central difference with one Richardson step: (4 D(h/2) - D(h)) / 3, error O(h^4)."""
    d1 = (fun(h) - fun(-h)) / (2 * h)
    d2 = (fun(h / 2) - fun(-h / 2)) / h
    return (4 * d2 - d1) / 3


def _run(D, X0, omega, K, safeguard):
    X, info = oracle.layout(D, X0, omega=omega, tol=0.0, max_iter=K, safeguard=safeguard)
    return X, info["trace"][:, 1].copy()


def test_sp_trees_match_scipy_and_are_trees():
    g, ln = _weighted()
    D, P = oracle.sp_trees(g.row_ptr, g.col_idx, ln)
    A = sp.csr_matrix((ln, g.col_idx, g.row_ptr), shape=(g.n, g.n))
    ref = shortest_path(A, method="D", directed=False)
    np.testing.assert_allclose(D, ref, rtol=1e-12)
    lenmap = {(int(u), int(v)): l for u, v, l in zip(np.repeat(np.arange(g.n), np.diff(g.row_ptr)), g.col_idx, ln)}
    Draw = np.array([oracle.sssp_rows(g.row_ptr, g.col_idx, [s], ln)[0] for s in range(g.n)])
    for s in range(g.n):
        for v in range(g.n):
            u = P[s, v]
            if v == s:
                assert u == -1
                continue
            assert u >= 0
            assert Draw[s, u] + lenmap[(u, v)] == Draw[s, v]
            # lowest-numbered among the predecessors that tie
            ties = [w for w in g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]] if Draw[s, w] + lenmap[(int(w), v)] == Draw[s, v]]
            assert u == min(ties)


def test_stress_grad_matches_finite_differences():
    g, X0 = inputs.grid16(0)
    D = oracle.apsp(g.row_ptr, g.col_idx)
    X = X0 * 10.0
    G = oracle.stress_grad(D, X)
    rng = np.random.default_rng(1)
    for _ in range(5):
        v = rng.standard_normal(X.shape)
        assert _fd(lambda h: oracle.stress(D, X + h * v)) == pytest.approx(np.sum(G * v), rel=1e-7)


@pytest.mark.parametrize("omega,safeguard", [(1.0, True), (1.5, True), (1.5, False), (2.5, True)])
def test_vjp_initial_placement_matches_finite_differences(omega, safeguard):
    g, ln = _weighted()
    D, _ = oracle.sp_trees(g.row_ptr, g.col_idx, ln)
    Dhop = oracle.apsp(g.row_ptr, g.col_idx)
    X0 = inputs.uniform_positions(g.n, 2, 5, hi=4.0)
    K = 12
    XK, acc = _run(D, X0, omega, K, safeguard)
    gX0, gD = oracle.layout_vjp(D, X0, omega, K, acc, oracle.stress_grad(Dhop, XK))
    rng = np.random.default_rng(2)
    for _ in range(4):
        v = rng.standard_normal(X0.shape)

        def f(h):
            X, a = _run(D, X0 + h * v, omega, K, safeguard)
            assert np.array_equal(a, acc)  # the same safeguard decisions
            return _loss(Dhop, X)

        assert _fd(f) == pytest.approx(np.sum(gX0 * v), rel=1e-6, abs=1e-9 * np.abs(gX0).sum())
    # invariance under translation and rotation of X0
    assert np.abs(gX0.sum(0)).max() <= 1e-9 * np.abs(gX0).sum()
    torque = np.sum(X0[:, 0] * gX0[:, 1] - X0[:, 1] * gX0[:, 0])
    assert abs(torque) <= 1e-9 * np.sum(np.abs(X0) * np.abs(gX0[:, ::-1]))


def test_vjp_distance_matches_finite_differences():
    g, ln = _weighted()
    D, _ = oracle.sp_trees(g.row_ptr, g.col_idx, ln)
    Dhop = oracle.apsp(g.row_ptr, g.col_idx)
    X0 = inputs.uniform_positions(g.n, 2, 6, hi=4.0)
    K, omega = 10, 1.5
    XK, acc = _run(D, X0, omega, K, True)
    _, gD = oracle.layout_vjp(D, X0, omega, K, acc, oracle.stress_grad(Dhop, XK))
    np.testing.assert_array_equal(gD, gD.T)
    rng = np.random.default_rng(3)
    for _ in range(6):
        s, t = sorted(rng.choice(g.n, 2, replace=False))

        def f(h):
            D2 = D.copy()
            D2[s, t] = D2[t, s] = D[s, t] + h
            X, a = _run(D2, X0, omega, K, True)
            assert np.array_equal(a, acc)
            return _loss(Dhop, X)

        assert _fd(f) == pytest.approx(gD[s, t], rel=1e-6, abs=1e-9 * np.abs(gD).max())


def test_edge_grad_matches_finite_differences():
    g, ln = _weighted()
    D, P = oracle.sp_trees(g.row_ptr, g.col_idx, ln)
    Dhop = oracle.apsp(g.row_ptr, g.col_idx)
    X0 = inputs.uniform_positions(g.n, 2, 7, hi=4.0)
    K, omega = 10, 1.5
    XK, acc = _run(D, X0, omega, K, True)
    _, gD = oracle.layout_vjp(D, X0, omega, K, acc, oracle.stress_grad(Dhop, XK))
    glen = oracle.edge_grad(g.row_ptr, g.col_idx, P, gD)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    rng = np.random.default_rng(4)
    checked = 0
    for e in rng.permutation(len(ln)):
        u, v = int(src[e]), int(g.col_idx[e])
        if u > v:
            continue
        twin = np.flatnonzero((src == v) & (g.col_idx == u))[0]
        assert glen[e] == glen[twin]
        def f(h):
            l2 = ln.copy()
            l2[e] += h
            l2[twin] += h
            D2, P2 = oracle.sp_trees(g.row_ptr, g.col_idx, l2)
            assert np.array_equal(P2, P)  # the same shortest paths
            X2, a2 = _run(D2, X0, omega, K, True)
            assert np.array_equal(a2, acc)
            return _loss(Dhop, X2)

        assert _fd(f) == pytest.approx(glen[e], rel=1e-6, abs=1e-9 * np.abs(glen).max())
        checked += 1
        if checked == 6:
            break
    # an edge on no shortest path gets 0
    used = np.zeros(len(ln), dtype=bool)
    for s in range(g.n):
        for t in range(s + 1, g.n):
            w = t
            while w != s:
                u = P[s, w]
                used |= ((src == u) & (g.col_idx == w)) | ((src == w) & (g.col_idx == u))
                w = u
    assert np.all(glen[~used] == 0.0)
