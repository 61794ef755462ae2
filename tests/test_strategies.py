"""Relaxation strategies of Sec. 5.2 (schedule, probabilistic, enumerating,
per-vertex factors): host validation and GPU parity with the oracle, and runs
resumed from their returned placement (iter_offset).

GPU trace column 3 holds the paper's factor used; the oracle's column 5.
Tolerances as in test_gpu_parity.py (1e-4 * diam per iteration), the
comparison of a run ending at the first decision the oracle took inside the
FP32 rounding band (safeguard: |f(X~) - f(X^H)| within 64 * 2^-24 of its term
scale; enumerating: the best and second-best candidates within that band).
"""
import numpy as np
import pytest

import oracle
from fixtures import ppi_fig4a
from lockstep import check_safeguard_lockstep
from paper_1711_01228_amd import binding as b
from paper_1711_01228_amd import inputs

AMBIG = 64 * 2.0 ** -24


@pytest.mark.parametrize("kw,msg", [
    (dict(strategy=7), "strategy"),
    (dict(strategy=b.SL_OMEGA_SCHEDULE), "needs omega_schedule"),
    (dict(strategy=b.SL_OMEGA_SCHEDULE, omega_schedule=np.array([1.5, 0.0, 1.2])), "outside"),
    (dict(strategy=b.SL_OMEGA_FIXED, omega_schedule=np.array([1.5, 1.5, 1.5])), "only read"),
    (dict(strategy=b.SL_OMEGA_ENUM, omega_vertex=1234), "per-vertex"),
])
def test_strategy_validation(kw, msg):
    o = b.make_options(max_iter=3, **kw)
    assert b.sl_validate_status(inputs.grid_graph(3, 3), o) == b.SL_EINVAL
    assert msg in b.last_error()


def _ppi():
    n, edges, _ = ppi_fig4a()
    return inputs.to_csr(n, edges)


def _compare(g, X0, iters, dim=2, gpu_kw=None, orc_kw=None, enum=False):
    import torch

    D = oracle.apsp(g.row_ptr, g.col_idx)
    Xo, io = oracle.layout(D, X0, tol=0.0, max_iter=iters, trace_positions=True, **orc_kw)
    X = torch.tensor(X0.astype(np.float32), device="cuda")
    with b.Plan(g, dim) as plan:
        ig = plan.run(X, tol=0.0, max_iter=iters, trace=True, trace_positions=True, **gpu_kw)
    assert ig["iterations"] == io["iterations"] == iters
    tg, to = ig["trace"], io["trace"]
    Pg, Po = ig["positions"].astype(np.float64), io["positions"]
    compared = 0
    for k in range(iters):
        amb = (abs(to[k, 6]) <= AMBIG * to[k, 7]) if enum else (abs(to[k, 2]) <= AMBIG * to[k, 3])
        same = (tg[k, 1] == to[k, 1]) and (np.isnan(to[k, 5]) or tg[k, 3] == to[k, 5])
        if not same:
            assert amb, (k, tg[k], to[k])
            break
        diam = float(np.linalg.norm(Po[k].max(0) - Po[k].min(0)))
        assert np.abs(Pg[k] - Po[k]).max() <= 1e-4 * diam, k
        compared += 1
    # every iteration, from the GPU's own iterate
    check_safeguard_lockstep(D, X0, ig, omega_vertex=orc_kw.get("omega_vertex"), enumerate=enum)
    return compared, ig, io


@pytest.mark.gpu
def test_probabilistic_strategy_matches_oracle():
    # the library draws the factors itself (SplitMix64 of the seed and the
    # iteration number); the oracle's own generator gives the same sequence
    g, X0 = inputs.grid16(3)
    sched = 1.0 + oracle.auto_factors(11, 0, 120)
    compared, ig, io = _compare(g, X0, 120, gpu_kw=dict(strategy="auto", seed=11),
                                orc_kw=dict(omega_schedule=sched))
    assert compared >= 80
    np.testing.assert_array_equal(ig["trace"][:, 3], sched - 1.0)  # every draw, also past the compared part


@pytest.mark.gpu
@pytest.mark.parametrize("kind", ["fixed", "schedule", "auto", "fixed_unordered"])
def test_resume_with_iter_offset_equals_one_run(kind):
    """k iterations, then k more from the returned placement with iter_offset
    = k, equal 2k iterations in one call bit for bit (the schedule and the
    probabilistic draws continue where the first call stopped)."""
    import torch

    g, X0 = inputs.grid16(6)
    k = 17
    sched = 1.0 + 0.25 * (np.arange(2 * k) % 7)  # 1.0 .. 2.5, factors of 1 included
    kw = {"fixed": dict(omega=1.7), "schedule": dict(strategy="schedule", omega_schedule=sched),
          "auto": dict(strategy="auto", seed=2024), "fixed_unordered": dict(omega=1.7, sym_force=True)}[kind]
    X1 = torch.tensor(X0.astype(np.float32), device="cuda")
    X2 = X1.clone()
    with b.Plan(g, 2) as plan:
        one = plan.run(X1, tol=0.0, max_iter=2 * k, trace=True, **kw)
        a = plan.run(X2, tol=0.0, max_iter=k, trace=True, **kw)
        c = plan.run(X2, tol=0.0, max_iter=k, trace=True, iter_offset=k, **kw)
    np.testing.assert_array_equal(X1.cpu().numpy(), X2.cpu().numpy())
    np.testing.assert_array_equal(one["trace"], np.concatenate([a["trace"], c["trace"]]))
    assert one["rejected"] == a["rejected"] + c["rejected"]
    if kind == "auto":  # the draws of iterations k .. 2k-1, not a restart of the sequence
        np.testing.assert_array_equal(c["trace"][:, 3], oracle.auto_factors(2024, k, k))
        assert not np.array_equal(c["trace"][:, 3], a["trace"][:, 3])


@pytest.mark.gpu
def test_schedule_of_ones_is_algorithm1_on_gpu():
    import torch

    g, X0 = inputs.grid16(4)
    X1 = torch.tensor(X0.astype(np.float32), device="cuda")
    X2 = X1.clone()
    with b.Plan(g, 2) as plan:
        plan.run(X1, omega=1.0, tol=0.0, max_iter=30)
        plan.run(X2, tol=0.0, max_iter=30, strategy="schedule", omega_schedule=np.ones(30))
    np.testing.assert_array_equal(X1.cpu().numpy(), X2.cpu().numpy())


@pytest.mark.gpu
@pytest.mark.parametrize("dim", [2, 3])
def test_enumerating_strategy_matches_oracle(dim):
    g = _ppi()
    X0 = inputs.uniform_positions(g.n, dim, seed=21)
    compared, ig, io = _compare(g, X0, 25, dim=dim, gpu_kw=dict(strategy="enum"), orc_kw=dict(enumerate=True),
                                enum=True)
    assert compared >= 10
    picks = io["trace"][:, 5]
    assert np.any(picks > 0.5)  # the argmin moves away from the small factors at times


@pytest.mark.gpu
def test_per_vertex_factors_match_oracle():
    import torch

    g = inputs.erdos_renyi(129, 400, 5)
    X0 = inputs.uniform_positions(g.n, 2, seed=9, hi=10.0)
    w = 1.0 + np.random.default_rng(4).uniform(0.0, 1.0, size=g.n)
    wt = torch.tensor(w.astype(np.float32), device="cuda")
    compared, ig, io = _compare(g, X0, 40, gpu_kw=dict(omega_vertex=wt),
                                orc_kw=dict(omega_vertex=w.astype(np.float32).astype(np.float64)))
    assert compared >= 30
    assert np.all(np.isnan(ig["trace"][:, 3]))
