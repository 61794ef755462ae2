"""The force pass over unordered pairs against the pass over all ordered
pairs: the same sums in another order.

One Jacobi step from the same start: max |x^sym - x^ordered| <= 2e-6 * diam
(both sum FP32 pair terms; the unordered pass adds each column's terms over
512 rows in FP32 before FP64).  Ragged sizes (n_pad not a multiple of the
512-row panel), tiny graphs, a disconnected graph with isolated vertices
(unreachable pairs carry no weight), 2-D and 3-D, hop counts and edge lengths.
The unordered pass is the default in 2-D from n_pad = 32768 (Jacobi step, no
stress trace); SL_FLAG_SYM_FORCE and SL_FLAG_ORDERED_FORCE pick either pass.
"""
import numpy as np
import pytest

from paper_1711_01228_amd import inputs

pytestmark = pytest.mark.gpu


def dev(X):
    import torch

    return torch.tensor(np.asarray(X, dtype=np.float32), device="cuda").contiguous()


def diam(X):
    return float(np.linalg.norm(X.max(0) - X.min(0)))


def graphs():
    return {
        "path2": inputs.to_csr(2, [(0, 1)]),
        "grid16": inputs.grid16(0)[0],
        "ragged_129": inputs.erdos_renyi(129, 400, 5),
        "tree700": inputs.random_tree(700, 3),
        "ba3000": inputs.barabasi_albert(3000, 3, 11),
        "er5000": inputs.erdos_renyi(5000, 15000, 2),
        "disconnected_600": disconnected(),
    }


def disconnected():
    # two components (a tree of 300 and a cycle of 200) and 100 isolated vertices
    t = inputs.random_tree(300, 8)
    edges = [(u, v) for u, v in t.edges()] + [(300 + k, 300 + (k + 1) % 200) for k in range(200)]
    return inputs.to_csr(600, edges)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("name", sorted(graphs()))
def test_unordered_pass_matches_ordered_pass(name, dim):
    from paper_1711_01228_amd import binding as b

    g = graphs()[name]
    print("case", name, dim, flush=True)
    X0 = inputs.uniform_positions(g.n, dim, seed=41, hi=float(np.sqrt(g.n)))
    with b.Plan(g, dim) as plan:
        Xs, Xd = dev(X0), dev(X0)
        plan.run(Xs, omega=1.0, tol=0.0, max_iter=1, sym_force=True)
        plan.run(Xd, omega=1.0, tol=0.0, max_iter=1, ordered_force=True)
        err = np.abs(Xs.cpu().numpy().astype(np.float64) - Xd.cpu().numpy()).max()
        assert err <= 2e-6 * diam(X0), err
        if name == "disconnected_600":  # isolated vertices have no pair with weight: they stay
            np.testing.assert_array_equal(Xs.cpu().numpy()[500:], X0[500:].astype(np.float32))
        # a few steps with extrapolation and the safeguard stay together too
        Xs, Xd = dev(X0), dev(X0)
        ts = plan.run(Xs, omega=1.5, tol=0.0, max_iter=10, trace=True, sym_force=True)["trace"]
        td = plan.run(Xd, omega=1.5, tol=0.0, max_iter=10, trace=True, ordered_force=True)["trace"]
        if np.array_equal(ts[:, 1], td[:, 1]):
            assert np.abs(Xs.cpu().numpy() - Xd.cpu().numpy()).max() <= 1e-5 * diam(Xd.cpu().numpy())


def test_unordered_pass_is_bitwise_repeatable():
    from paper_1711_01228_amd import binding as b

    g, X0 = inputs.grid16(2)
    with b.Plan(g, 2) as plan:
        outs = []
        for _ in range(3):
            X = dev(X0)
            plan.run(X, omega=1.5, tol=0.0, max_iter=25, sym_force=True)
            outs.append(X.cpu().numpy())
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])


def test_unordered_pass_is_refused_where_it_does_not_apply():
    from paper_1711_01228_amd import binding as b

    g, X0 = inputs.grid16(0)
    with b.Plan(g, 2) as plan:
        for kw in ({"trace_stress": True}, {"trace_stress": True, "ordering": "exact"}):
            with pytest.raises(b.SlError) as e:
                plan.run(dev(X0), max_iter=2, sym_force=True, **kw)
            assert e.value.status == b.SL_ENOTSUP


@pytest.mark.parametrize("dim", [2, 3])
def test_unordered_pass_on_edge_length_plan(dim):
    # FP32 path lengths (edge lengths 1 +- 0.3): 1/d by the reciprocal instruction on both passes
    from paper_1711_01228_amd import binding as b

    g = inputs.largest_component(inputs.erdos_renyi(700, 2100, 17))
    ln = (1.0 + np.random.default_rng(18).uniform(-0.3, 0.3, g.num_edges)).astype(np.float32)
    gw = inputs.to_csr(g.n, g.edges(), ln)
    X0 = inputs.uniform_positions(g.n, dim, seed=19, hi=float(np.sqrt(g.n)))
    print("case weighted", g.n, dim, flush=True)
    with b.Plan(gw, dim) as plan:
        Xs, Xd = dev(X0), dev(X0)
        plan.run(Xs, omega=1.0, tol=0.0, max_iter=1, sym_force=True)
        plan.run(Xd, omega=1.0, tol=0.0, max_iter=1, ordered_force=True)
        err = np.abs(Xs.cpu().numpy().astype(np.float64) - Xd.cpu().numpy()).max()
        assert err <= 2e-6 * diam(X0), err
        ms = plan.profile(dev(X0), omega=1.5, reps=1)
        assert ms["force_sym"] > 0.0 and ms["force_safeguard_sym"] > 0.0


def lengths_graph(n, seed):
    g = inputs.erdos_renyi(n, 4 * n, seed)
    ln = (1.0 + np.random.default_rng(seed + 1).uniform(-0.1, 0.1, g.num_edges)).astype(np.float32)
    return inputs.to_csr(g.n, g.edges(), ln)


DEFAULT_CASES = {
    "grid16": lambda: inputs.grid_graph(16, 16),              # n_pad 256: the ordered pass is faster
    "ba16384": lambda: inputs.barabasi_albert(16384, 3, 64),  # n_pad 16384: unordered only for fused runs
    "ba24576": lambda: inputs.barabasi_albert(24576, 3, 61),  # n_pad 24576: the unordered one
    "er8192_lengths": lambda: lengths_graph(8192, 62),        # edge lengths: ordered below n_pad 16384
    "er16384_lengths": lambda: lengths_graph(16384, 63),      # and unordered from there
}


# (graph, dim, omega of the run, the pass it takes by default)
@pytest.mark.parametrize("name,dim,omega,expect", [
    ("grid16", 2, 1.5, "ordered"), ("grid16", 3, 1.5, "ordered"),
    ("ba16384", 2, 1.0, "ordered"), ("ba16384", 2, 1.5, "sym"), ("ba16384", 3, 1.5, "sym"),
    ("ba24576", 2, 1.0, "sym"), ("ba24576", 3, 1.0, "sym"),
    ("er8192_lengths", 2, 1.5, "ordered"), ("er16384_lengths", 2, 1.5, "sym"), ("er16384_lengths", 3, 1.0, "sym"),
])
def test_default_force_pass_by_size_and_dim(name, dim, omega, expect):
    from paper_1711_01228_amd import binding as b

    g = DEFAULT_CASES[name]()
    X0 = inputs.uniform_positions(g.n, dim, seed=43, hi=float(np.sqrt(g.n)))
    print("case default pass", name, dim, flush=True)
    with b.Plan(g, dim) as plan:
        outs = {}
        for kind, kw in (("default", {}), ("sym", {"sym_force": True}), ("ordered", {"ordered_force": True})):
            X = dev(X0)
            plan.run(X, omega=omega, tol=0.0, max_iter=6, **kw)
            outs[kind] = X.cpu().numpy()
        with pytest.raises(b.SlError) as e:
            plan.run(dev(X0), max_iter=2, sym_force=True, ordered_force=True)
        assert e.value.status == b.SL_EINVAL
    np.testing.assert_array_equal(outs["default"], outs[expect])
