"""torch.autograd integration: a differentiable batched power-flow solve.

``solve(net, p, q, vm_set)`` returns the converged complex bus voltages; its
backward pass runs the library's adjoint (one transposed-Jacobian GMRES solve
per scenario, pf_tx_adjoint) to map dL/dV onto dL/dP (Theta buses) and dL/dQ
(PQ buses).  Injections that the solve does not read (the slack's P and Q, the
Q of PV buses) get zero gradient; the voltage set-points are not
differentiated.

A gradient is only meaningful for a scenario whose forward solve converged
(the implicit function theorem needs F(x, P, Q) = 0) and whose adjoint GMRES
solve met its tolerance.  By default the backward pass raises
``NonConvergedGradient`` when either fails for any scenario; with
``on_failure="zero"`` it warns instead and returns zero gradient rows for the
failed scenarios.
"""
from __future__ import annotations

import warnings

import torch

from .pf import TxNetwork


class NonConvergedGradient(RuntimeError):
    """The forward solve or the adjoint solve of some scenario did not converge."""

    def __init__(self, msg: str, forward_failed: list[int], adjoint_failed: list[int]):
        super().__init__(msg)
        self.forward_failed = forward_failed
        self.adjoint_failed = adjoint_failed


class _PFSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, p, q, vm_set, net, opts, adj_opts, on_failure):
        res = net.solve(p.detach().contiguous(), q.detach().contiguous(), vm_set.detach().contiguous(), **opts)
        ctx.net = net
        ctx.adj_opts = adj_opts
        ctx.on_failure = on_failure
        ctx.save_for_backward(res.v, res.converged)
        ctx.mark_non_differentiable(res.converged)
        return res.v, res.converged

    @staticmethod
    def backward(ctx, grad_v, grad_conv):
        v, conv = ctx.saved_tensors
        if grad_v is None:
            return None, None, None, None, None, None, None
        gp, gq, _, ok = ctx.net.adjoint(v, grad_v.contiguous(), **ctx.adj_opts)
        fwd_bad = (conv == 0).nonzero().flatten().tolist()
        adj_bad = (ok == 0).nonzero().flatten().tolist()
        if fwd_bad or adj_bad:
            msg = (f"power-flow gradient undefined for scenarios: forward solve not converged {fwd_bad[:16]}, "
                   f"adjoint GMRES not converged {adj_bad[:16]}")
            if ctx.on_failure == "raise":
                raise NonConvergedGradient(msg, fwd_bad, adj_bad)
            warnings.warn(msg + " (their gradient rows are set to zero)", RuntimeWarning, stacklevel=2)
            bad = (conv == 0) | (ok == 0)
            gp = gp.masked_fill(bad[:, None], 0.0)
            gq = gq.masked_fill(bad[:, None], 0.0)
        return gp, gq, None, None, None, None, None


def solve(net: TxNetwork, p: torch.Tensor, q: torch.Tensor, vm_set: torch.Tensor, *,
          adjoint_opts: dict | None = None, on_failure: str = "raise", **opts):
    """Differentiable solve: returns (v complex128 (B, n), converged uint8 (B,)).

    ``opts`` go to the forward solve (pf_tx_solve); ``adjoint_opts`` to the
    backward one (pf_tx_adjoint; by default the forward's GMRES restart
    options).  ``on_failure``: "raise" or "zero" (see the module docstring).
    """
    if on_failure not in ("raise", "zero"):
        raise ValueError("on_failure must be 'raise' or 'zero'")
    if adjoint_opts is None:
        adjoint_opts = {k: v for k, v in opts.items() if k in ("gmres_restart", "gmres_max_restarts")}
    return _PFSolve.apply(p, q, vm_set, net, opts, dict(adjoint_opts), on_failure)
