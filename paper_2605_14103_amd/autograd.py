"""torch.autograd integration: a differentiable batched power-flow solve.

``solve(net, p, q, vm_set)`` returns the converged complex bus voltages; its
backward pass runs the library's adjoint (one transposed-Jacobian GMRES solve
per scenario, pf_tx_adjoint) to map dL/dV onto dL/dP (Theta buses) and dL/dQ
(PQ buses).  Injections that the solve does not read (the slack's P and Q, the
Q of PV buses) get zero gradient; the voltage set-points are not
differentiated.
"""
from __future__ import annotations

import torch

from .pf import TxNetwork


class _PFSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, p, q, vm_set, net, opts):
        res = net.solve(p.detach().contiguous(), q.detach().contiguous(), vm_set.detach().contiguous(), **opts)
        ctx.net = net
        ctx.adj_opts = {k: v for k, v in opts.items() if k in ("gmres_restart", "gmres_max_restarts")}
        ctx.save_for_backward(res.v)
        ctx.mark_non_differentiable(res.converged)
        return res.v, res.converged

    @staticmethod
    def backward(ctx, grad_v, grad_conv):
        (v,) = ctx.saved_tensors
        if grad_v is None:
            return None, None, None, None, None
        gp, gq, _, _ = ctx.net.adjoint(v, grad_v.contiguous(), **ctx.adj_opts)
        return gp, gq, None, None, None


def solve(net: TxNetwork, p: torch.Tensor, q: torch.Tensor, vm_set: torch.Tensor, **opts):
    """Differentiable solve: returns (v complex128 (B, n), converged uint8 (B,))."""
    return _PFSolve.apply(p, q, vm_set, net, opts)
