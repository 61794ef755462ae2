"""The allocation-free batched layout against the batched plan on the GPU.

sl_batch_layout_noalloc runs the kernels of sl_batch_plan_create +
sl_batch_plan_run (untuned defaults) out of the library's static device array,
so each graph's placement and results must equal the plan path's bit for bit
(which is within the floating-point bar of the batched parity tests, 1e-4 of the
layout diameter, by a wide margin).  Two calls in a row, the second with a
smaller batch, check that the shared array is re-initialized between calls.
"""
import numpy as np
import pytest

from paper_1711_01228_amd import binding as b
from paper_1711_01228_amd import inputs

pytestmark = pytest.mark.gpu


def batch_a():
    gs = [inputs.grid_graph(16, 16), inputs.largest_component(inputs.erdos_renyi(300, 600, 21)),
          inputs.random_tree(500, 22), inputs.near_square_grid(700),
          inputs.largest_component(inputs.erdos_renyi(1000, 2000, 23)), inputs.to_csr(1, []),
          inputs.to_csr(2, [(0, 1)])]
    return gs


def batch_b():
    return [inputs.grid_graph(8, 8), inputs.random_tree(100, 31), inputs.largest_component(inputs.erdos_renyi(200, 400, 32))]


def starts(gs, dim, seed):
    return np.concatenate([inputs.uniform_positions(g.n, dim, seed + k) for k, g in enumerate(gs)]).astype(np.float32)


def plan_path(gs, X0, dim, omega, tol, max_iter):
    import torch

    X = torch.tensor(X0, device="cuda")
    with b.BatchPlan(gs, dim) as plan:
        tot, per = plan.run(X, omega=omega, tol=tol, max_iter=max_iter)
    return X.cpu().numpy(), tot, per


def noalloc_path(gs, X0, dim, omega, tol, max_iter):
    import torch

    args = b.BatchArgs(gs)
    X = torch.tensor(X0, device="cuda")
    opt = b.make_options(dim, omega, tol, max_iter, True)
    tot, per = b.sl_batch_layout_noalloc(args, X.data_ptr(), opt)
    torch.cuda.synchronize()
    return X.cpu().numpy(), tot, per


def check_equal(gs, got, ref):
    Xn, tn, pn = got
    Xp, tp, pp = ref
    assert np.array_equal(Xn, Xp), "placements differ from the batched plan's"
    off = 0
    for k, g in enumerate(gs):
        x = Xp[off:off + g.n].astype(np.float64)
        diam = float(np.linalg.norm(x.max(0) - x.min(0))) if g.n else 0.0
        assert np.abs(Xn[off:off + g.n] - Xp[off:off + g.n]).max(initial=0.0) <= 1e-4 * diam
        off += g.n
        for key in ("iterations", "converged", "rejected", "residual", "stress"):
            assert pn[k][key] == pp[k][key], (k, key, pn[k][key], pp[k][key])
    for key in ("iterations", "converged", "rejected", "residual"):
        assert tn[key] == tp[key], key
    assert np.isnan(tn["run_ms"]) and np.isnan(tn["plan_ms"])


@pytest.mark.parametrize("dim", [2, 3])
def test_noalloc_equals_batched_plan_two_calls(dim):
    import torch

    torch.cuda.set_device(0)
    ga, gb = batch_a(), batch_b()
    xa, xb = starts(ga, dim, 500), starts(gb, dim, 600)
    print("noalloc: dim %d, batch A %s, batch B %s" % (dim, [g.n for g in ga], [g.n for g in gb]), flush=True)
    ref_a = plan_path(ga, xa, dim, 1.5, 1e-3, 400)
    ref_b = plan_path(gb, xb, dim, 1.5, 1e-3, 400)
    check_equal(ga, noalloc_path(ga, xa, dim, 1.5, 1e-3, 400), ref_a)
    check_equal(gb, noalloc_path(gb, xb, dim, 1.5, 1e-3, 400), ref_b)  # smaller, right after


def test_noalloc_fixed_steps_and_no_safeguard():
    import torch

    torch.cuda.set_device(0)
    ga = batch_a()
    xa = starts(ga, 2, 700)
    for omega, sg in ((1.0, True), (2.5, False)):
        Xp, tp, pp = plan_path_opts(ga, xa, omega, sg)
        args = b.BatchArgs(ga)
        X = torch.tensor(xa, device="cuda")
        tn, pn = b.sl_batch_layout_noalloc(args, X.data_ptr(), b.make_options(2, omega, 0.0, 30, sg))
        assert np.array_equal(X.cpu().numpy(), Xp)
        assert [r["rejected"] for r in pn] == [r["rejected"] for r in pp]


def plan_path_opts(gs, X0, omega, sg):
    import torch

    X = torch.tensor(X0, device="cuda")
    with b.BatchPlan(gs, 2) as plan:
        tot, per = plan.run(X, omega=omega, tol=0.0, max_iter=30, safeguard=sg)
    return X.cpu().numpy(), tot, per


def test_noalloc_rejects_a_batch_beyond_its_scratch():
    import torch

    torch.cuda.set_device(0)
    gs = [inputs.grid_graph(32, 32)] * 17  # 17 distance blocks of 1 MiB > 16 MiB
    args = b.BatchArgs(gs)
    X = torch.zeros((args.n_total, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(b.SlError) as ei:
        b.sl_batch_layout_noalloc(args, X.data_ptr(), b.make_options(2, 1.5, 1e-3, 10, True))
    assert ei.value.status == b.SL_EINVAL and "SL_NOALLOC_SCRATCH_BYTES" in str(ei.value)
    # the next call on the same array still matches the plan path
    gb = batch_b()
    xb = starts(gb, 2, 800)
    check_equal(gb, noalloc_path(gb, xb, 2, 1.5, 1e-3, 400), plan_path(gb, xb, 2, 1.5, 1e-3, 400))
