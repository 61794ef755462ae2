"""torch.autograd functions over the library's reverse mode.

Argument marshalling only: the forward iterations, the adjoint passes and the
shortest-path routing of edge-length derivatives all run in the HIP library
(``sl_plan_unroll``, ``sl_plan_unroll_backward``, ``sl_plan_stress_grad``).

    lay = DifferentiableLayout(g, dim=2)          # g: graph with edge lengths
    X = unrolled_layout(X0, lengths, lay, omega=1.5, iters=100, ckpt_every=10)
    loss = stress_loss(X, lay)                    # eq. 1 against hop distances
    loss.backward()                               # X0.grad, lengths.grad

``lengths`` holds one length per undirected edge, in the order of
``g.edges()`` (pairs i < j).  The derivative holds the safeguard decisions of
the forward run fixed (they are piecewise constant in the inputs).
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding
from .inputs import Graph, to_csr


class DifferentiableLayout:
    """An edge-length plan (d = shortest-path lengths) and a hop-count plan for
    the stress loss, over the same graph.  One forward/backward pair at a
    time: a forward replaces the tape of the previous one."""

    def __init__(self, g: Graph, dim: int = 2, lengths=None):
        self.n, self.dim = int(g.n), int(dim)
        self.edges = g.edges()
        m = len(self.edges)
        init = np.ones(m, dtype=np.float32) if lengths is None else np.asarray(lengths, dtype=np.float32)
        gw = to_csr(g.n, self.edges, init)
        self.row_ptr, self.col_idx = gw.row_ptr, gw.col_idx
        src = np.repeat(np.arange(g.n), np.diff(gw.row_ptr))
        # CSR entry of every undirected edge in both directions
        key = src.astype(np.int64) * g.n + gw.col_idx
        order = np.argsort(key)
        fwd = self.edges[:, 0].astype(np.int64) * g.n + self.edges[:, 1]
        bwd = self.edges[:, 1].astype(np.int64) * g.n + self.edges[:, 0]
        self.entry_fwd = order[np.searchsorted(key[order], fwd)]
        self.entry_bwd = order[np.searchsorted(key[order], bwd)]
        self.nnz = int(gw.nnz)
        self.plan = binding.Plan(gw, dim)
        self.hop_plan = binding.Plan(to_csr(g.n, self.edges), dim)

    def csr_lengths(self, lengths) -> np.ndarray:
        ln = np.asarray(lengths, dtype=np.float32).reshape(-1)
        out = np.empty(self.nnz, dtype=np.float32)
        out[self.entry_fwd] = ln
        out[self.entry_bwd] = ln
        return out

    def set_lengths(self, lengths) -> None:
        self.plan.set_lengths(self.csr_lengths(lengths))

    def close(self):
        self.plan.close()
        self.hop_plan.close()


class UnrolledLayout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X0, lengths, layout, omega, iters, ckpt_every, safeguard, force):
        if lengths is not None:
            layout.set_lengths(lengths.detach().float().cpu().numpy())
        X = X0.detach().to(device="cuda", dtype=torch.float32).contiguous().clone()
        info = layout.plan.unroll(X, omega=omega, iters=iters, ckpt_every=ckpt_every, safeguard=safeguard,
                                  sym_force=force == "unordered", ordered_force=force == "ordered")
        ctx.layout = layout
        ctx.has_len = lengths is not None
        ctx.info = info
        return X

    @staticmethod
    def backward(ctx, gX):
        lay = ctx.layout
        G = gX.detach().to(torch.float32).contiguous()
        gX0 = torch.empty_like(G)
        glen_csr = None
        if ctx.has_len and ctx.needs_input_grad[1]:
            glen_csr = torch.empty(lay.nnz, dtype=torch.float32, device=G.device)
        lay.plan.unroll_backward(G, gX0, glen_csr)
        glen = None
        if glen_csr is not None:
            glen = glen_csr[torch.as_tensor(lay.entry_fwd, device=G.device)]
        return gX0, glen, None, None, None, None, None, None


class StressLoss(torch.autograd.Function):
    """f(X) of eq. 1 against hop distances, as a float64 scalar."""

    @staticmethod
    def forward(ctx, X, layout):
        Xc = X.detach().to(torch.float32).contiguous()
        G = torch.empty_like(Xc)
        f = layout.hop_plan.stress_grad(Xc, G)
        ctx.save_for_backward(G)
        return torch.tensor(f, dtype=torch.float64, device=X.device)

    @staticmethod
    def backward(ctx, gf):
        (G,) = ctx.saved_tensors
        return G * gf.to(G.dtype), None


def unrolled_layout(X0, lengths, layout: DifferentiableLayout, omega=1.5, iters=100, ckpt_every=10,
                    safeguard=True, force="default"):
    """force: the force pass of the forward and backward, "default" (the
    library's choice by size), "unordered" (once per unordered pair) or
    "ordered" (every ordered pair)."""
    if force not in ("default", "unordered", "ordered"):
        raise ValueError("force must be 'default', 'unordered' or 'ordered'")
    return UnrolledLayout.apply(X0, lengths, layout, float(omega), int(iters), int(ckpt_every), bool(safeguard),
                                force)


def stress_loss(X, layout: DifferentiableLayout):
    return StressLoss.apply(X, layout)
