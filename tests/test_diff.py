"""Reverse mode on the GPU (unrolled Jacobi-SOR iterations, edge lengths
through the shortest paths) against the FP64 oracle's adjoint, finite
differences of the GPU forward, and invariants.

Tolerances (FP32 forward and adjoint passes, FP64 accumulation):
  * dL/dX0 and dL/dlen vs the oracle: ||g - g_orc|| <= 1e-3 ||g_orc|| (the
    oracle runs the same iterations from the same start with the decisions the
    GPU took, in FP64, on its own shortest paths)
  * at n = 1000: directional derivatives against Richardson central
    differences of the FP64 forward (same decisions, same trees): 5e-3
    relative (central differences of the FP32 forward are dominated by its
    rounding and are not used)
  * translation invariance sum_i dL/dx0_i = 0 and zero torque: within 1e-4 of
    sum |x0_i| |dL/dx0_i|
"""
import numpy as np
import pytest

import oracle
from paper_1711_01228_amd import inputs

pytestmark = pytest.mark.gpu


def _b():
    from paper_1711_01228_amd import binding

    return binding


def dev(X):
    import torch

    return torch.tensor(np.asarray(X, dtype=np.float32), device="cuda").contiguous()


def weighted_er(n, mean_degree, seed, spread=0.1):
    g = inputs.largest_component(inputs.erdos_renyi(n, n * mean_degree // 2, seed))
    rng = np.random.default_rng(seed + 7)
    e = g.edges()
    return g, (1.0 + rng.uniform(-spread, spread, len(e))).astype(np.float32)


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_unroll_equals_run_and_hop_gradient_matches_oracle():
    b = _b()
    g, X0 = inputs.grid16(5)
    K, omega = 20, 1.5
    D = oracle.apsp(g.row_ptr, g.col_idx)
    with b.Plan(g, 2) as plan:
        Xr = dev(X0)
        plan.run(Xr, omega=omega, tol=0.0, max_iter=K)
        X = dev(X0)
        info = plan.unroll(X, omega=omega, iters=K, ckpt_every=6)
        np.testing.assert_array_equal(X.cpu().numpy(), Xr.cpu().numpy())
        G = dev(np.zeros_like(X0))
        f = plan.stress_grad(X, G)
        gX0 = dev(np.zeros_like(X0))
        plan.unroll_backward(G, gX0)
        gX0 = gX0.cpu().numpy().astype(np.float64)
    XK = X.cpu().numpy().astype(np.float64)
    assert f == pytest.approx(oracle.stress(D, XK), rel=1e-5)
    np.testing.assert_allclose(G.cpu().numpy(), oracle.stress_grad(D, XK), rtol=0,
                               atol=1e-4 * np.abs(oracle.stress_grad(D, XK)).max())
    _, io = oracle.layout(D, X0, omega=omega, tol=0.0, max_iter=K)
    ref, _ = oracle.layout_vjp(D, X0, omega, K, io["trace"][:, 1], oracle.stress_grad(D, XK))
    assert _relerr(gX0, ref) <= 1e-3, _relerr(gX0, ref)
    print("info", info, "relerr", _relerr(gX0, ref), flush=True)


# "unordered": the force pass the differentiation workload takes at its size
# (once per unordered pair, FP32 edge-length distances), forward and backward
@pytest.mark.parametrize("force", ["default", "unordered"])
@pytest.mark.parametrize("omega,safeguard", [(1.0, True), (1.5, True), (1.5, False)])
def test_weighted_gradients_match_oracle(omega, safeguard, force):
    import torch

    from paper_1711_01228_amd import autograd as ag

    g, ln = weighted_er(200, 6, 11)
    X0 = inputs.uniform_positions(g.n, 2, 12, hi=6.0)
    K = 20
    lay = ag.DifferentiableLayout(g, 2, ln)
    try:
        X0t = dev(X0).requires_grad_(True)
        lt = torch.tensor(ln, device="cuda", requires_grad=True)
        print("case weighted gradients omega", omega, "safeguard", safeguard, force, flush=True)
        X = ag.unrolled_layout(X0t, lt, lay, omega=omega, iters=K, ckpt_every=7, safeguard=safeguard, force=force)
        loss = ag.stress_loss(X, lay)
        loss.backward()
        gX0 = X0t.grad.cpu().numpy().astype(np.float64)
        glen = lt.grad.cpu().numpy().astype(np.float64)
        Pg = lay.plan.tree_rows(np.arange(g.n))
    finally:
        lay.close()
    # the oracle on its own shortest paths, with the GPU's decisions
    gw = inputs.to_csr(g.n, g.edges(), ln)
    D, P = oracle.sp_trees(gw.row_ptr, gw.col_idx, gw.edge_len.astype(np.float64))
    Dhop = oracle.apsp(g.row_ptr, g.col_idx)
    Xo, io = oracle.layout(D, X0, omega=omega, tol=0.0, max_iter=K, safeguard=safeguard)
    assert float(loss.detach()) == pytest.approx(oracle.stress(Dhop, Xo), rel=1e-4)
    gX0_ref, gD = oracle.layout_vjp(D, X0, omega, K, io["trace"][:, 1], oracle.stress_grad(Dhop, Xo))
    assert _relerr(gX0, gX0_ref) <= 1e-3, _relerr(gX0, gX0_ref)
    assert np.array_equal(Pg, P), "trees differ (a near-tie); see test_weighted for tree parity"
    glen_csr = oracle.edge_grad(gw.row_ptr, gw.col_idx, P, gD)
    # per undirected edge, in the order of g.edges()
    src = np.repeat(np.arange(gw.n), np.diff(gw.row_ptr))
    key = {(int(u), int(v)): k for k, (u, v) in enumerate(zip(src, gw.col_idx))}
    glen_ref = np.array([glen_csr[key[(int(u), int(v))]] for u, v in g.edges()])
    assert _relerr(glen, glen_ref) <= 1e-3, _relerr(glen, glen_ref)
    print("relerr X0 %.2e len %.2e" % (_relerr(gX0, gX0_ref), _relerr(glen, glen_ref)), flush=True)


def _fd(fun, h):
    """Central difference with one Richardson step, error O(h^4)."""
    d1 = (fun(h) - fun(-h)) / (2 * h)
    d2 = (fun(h / 2) - fun(-h / 2)) / h
    return (4 * d2 - d1) / 3


@pytest.mark.parametrize("force", ["default", "unordered"])
def test_gpu_gradient_vs_fp64_finite_differences_and_invariants(force):
    import torch

    from paper_1711_01228_amd import autograd as ag

    g, ln = weighted_er(1000, 8, 21)
    X0 = inputs.uniform_positions(g.n, 2, 22, hi=10.0)
    K, omega = 30, 1.5
    lay = ag.DifferentiableLayout(g, 2, ln)
    print("case finite differences", force, flush=True)
    try:
        X0t = dev(X0).requires_grad_(True)
        lt = torch.tensor(ln, device="cuda", requires_grad=True)
        loss = ag.stress_loss(ag.unrolled_layout(X0t, lt, lay, omega=omega, iters=K, ckpt_every=10, force=force),
                              lay)
        loss.backward()
        gX0 = X0t.grad.cpu().numpy().astype(np.float64)
        glen = lt.grad.cpu().numpy().astype(np.float64)
        info = lay.plan.unroll(dev(X0), omega=omega, iters=K, ckpt_every=10, sym_force=force == "unordered")
    finally:
        lay.close()
    # finite differences of the FP64 forward (the oracle), same decisions and trees
    gw = inputs.to_csr(g.n, g.edges(), ln)
    Dhop = oracle.apsp(g.row_ptr, g.col_idx)
    D, P = oracle.sp_trees(gw.row_ptr, gw.col_idx, gw.edge_len.astype(np.float64))
    _, io = oracle.layout(D, X0, omega=omega, tol=0.0, max_iter=K)
    assert io["rejected"] == info["rejected"]
    acc = io["trace"][:, 1].copy()

    def run(Dm, x0):
        X, i2 = oracle.layout(Dm, x0, omega=omega, tol=0.0, max_iter=K)
        assert np.array_equal(i2["trace"][:, 1], acc)
        return oracle.stress(Dhop, X)

    src = np.repeat(np.arange(gw.n), np.diff(gw.row_ptr))
    key = {(int(u), int(v)): k for k, (u, v) in enumerate(zip(src, gw.col_idx))}
    ent = np.array([key[(int(u), int(v))] for u, v in g.edges()])
    twin = np.array([key[(int(v), int(u))] for u, v in g.edges()])
    rng = np.random.default_rng(5)
    v = rng.standard_normal(X0.shape)
    fd = _fd(lambda h: run(D, X0 + h * v), 1e-4)
    assert fd == pytest.approx(np.sum(gX0 * v), rel=5e-3)
    u = rng.standard_normal(len(ln))

    def run_len(h):
        l2 = gw.edge_len.astype(np.float64).copy()
        l2[ent] += h * u
        l2[twin] += h * u
        D2, P2 = oracle.sp_trees(gw.row_ptr, gw.col_idx, l2)
        assert np.array_equal(P2, P)
        return run(D2, X0)

    fd = _fd(run_len, 1e-7)  # small enough that no shortest path changes
    assert fd == pytest.approx(np.sum(glen * u), rel=5e-3)
    scale = np.sum(np.abs(X0) * np.abs(gX0[:, ::-1]))
    assert np.abs(gX0.sum(0)).max() <= 1e-4 * np.abs(gX0).sum()
    assert abs(np.sum(X0[:, 0] * gX0[:, 1] - X0[:, 1] * gX0[:, 0])) <= 1e-4 * scale


def test_backward_without_tape_and_length_gradient_on_hop_plan_are_refused():
    b = _b()
    g, X0 = inputs.grid16(0)
    with b.Plan(g, 2) as plan:
        G = dev(np.zeros_like(X0))
        with pytest.raises(b.SlError):
            plan.unroll_backward(G, dev(np.zeros_like(X0)))
        X = dev(X0)
        plan.unroll(X, iters=3, ckpt_every=2)
        import torch

        with pytest.raises(b.SlError) as e:
            plan.unroll_backward(G, dev(np.zeros_like(X0)), torch.zeros(g.nnz, device="cuda"))
        assert e.value.status == b.SL_EINVAL


def test_full_size_gradient_invariants():
    """ER n = 16,384, mean degree 8, 100 iterations at omega = 1.5, checkpoints
    every 10: gradients finite, translation- and rotation-invariant.  At this
    size an edge-length plan takes the unordered force pass; the unrolled
    forward equals sl_plan_run bit for bit on it.  Along a random direction v of
    the start: over 20 iterations the unordered pass's adjoint equals the
    ordered pass's (pinned against FP64 finite differences of the oracle at
    n = 1,000), and over one iteration it equals the central difference of the
    forward itself.  A central difference over 100 iterations is no check here:
    the forward's FP32 rounding makes f noisy at ~1e-7 of its value, which
    swamps h (g . v) at every usable h."""
    import torch

    from paper_1711_01228_amd import autograd as ag

    n = 16384
    g = inputs.erdos_renyi(n, n * 4, inputs.workload_seed(5))
    rng = np.random.default_rng(inputs.workload_seed(5) + 1)
    ln = (1.0 + rng.uniform(-0.1, 0.1, g.num_edges)).astype(np.float32)
    X0 = inputs.uniform_positions(n, 2, inputs.workload_seed(5) + 2, 0.0, float(np.sqrt(n)))
    print("case er16384 diff", flush=True)
    lay = ag.DifferentiableLayout(g, 2, ln)
    try:
        X0t = dev(X0).requires_grad_(True)
        lt = torch.tensor(ln, device="cuda", requires_grad=True)
        loss = ag.stress_loss(ag.unrolled_layout(X0t, lt, lay, omega=1.5, iters=100, ckpt_every=10), lay)
        loss.backward()
        gX0 = X0t.grad.cpu().numpy().astype(np.float64)
        glen = lt.grad.cpu().numpy().astype(np.float64)
        Xa, Xb = dev(X0), dev(X0)
        lay.plan.run(Xa, omega=1.5, tol=0.0, max_iter=20)
        lay.plan.unroll(Xb, omega=1.5, iters=20, ckpt_every=10)
        np.testing.assert_array_equal(Xa.cpu().numpy(), Xb.cpu().numpy())

        v = np.random.default_rng(inputs.workload_seed(5) + 3).standard_normal(X0.shape)

        def adjoint(iters, force):
            x0 = dev(X0).requires_grad_(True)
            ag.stress_loss(ag.unrolled_layout(x0, lt.detach(), lay, omega=1.5, iters=iters, ckpt_every=10,
                                              force=force), lay).backward()
            return float(np.sum(x0.grad.cpu().numpy().astype(np.float64) * v))

        def forward(x0, iters):
            X = dev(x0)
            info = lay.plan.unroll(X, omega=1.5, iters=iters, ckpt_every=10)
            return lay.hop_plan.stress(X), info["rejected"]

        a_sym, a_ord = adjoint(20, "default"), adjoint(20, "ordered")
        a1 = adjoint(1, "default")
        h = 1e-2
        (fp, rp), (fm, rm) = forward(X0 + h * v, 1), forward(X0 - h * v, 1)
        fd1 = (fp - fm) / (2 * h)
        print("directional derivative, 20 iterations: unordered %.6e, ordered %.6e; one iteration: adjoint %.6e, "
              "central difference %.6e" % (a_sym, a_ord, a1, fd1), flush=True)
    finally:
        lay.close()
    assert a_sym == pytest.approx(a_ord, rel=1e-3)
    assert rp == rm
    assert fd1 == pytest.approx(a1, rel=3e-2)
    assert np.all(np.isfinite(gX0)) and np.all(np.isfinite(glen))
    assert np.abs(glen).max() > 0
    assert np.abs(gX0.sum(0)).max() <= 1e-4 * np.abs(gX0).sum()
    scale = np.sum(np.abs(X0) * np.abs(gX0[:, ::-1]))
    assert abs(np.sum(X0[:, 0] * gX0[:, 1] - X0[:, 1] * gX0[:, 0])) <= 1e-4 * scale
