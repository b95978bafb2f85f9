"""Oracle: branch-current loss and the dense adjoint of the Newton-Raphson solution.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Loss (a reading of the sensitivity workload): for every branch the from-end
current including its charging, I_f = (y_s + j b/2) V_f - y_s V_t, and
L = sum over branches of |I_f|^2, per scenario.

Sensitivity: the solved state x(P, Q) satisfies F(x, P, Q) = 0 with
F = [P_calc(x) - P ; Q_calc(x) - Q] (eq. (2)).  Differentiating,
J dx = [dP ; dQ], so dL/d[P ; Q] = lambda with J^T lambda = dL/dx, where J is
the polar Jacobian of eq. (4) at the converged point.  The oracle forms J
densely and solves with LAPACK.
"""
from __future__ import annotations

import numpy as np

from . import nr


def branch_currents(grid, V):
    """From-end branch currents I_f [n_branch, ...] for voltages V [n_bus, ...]."""
    ys = 1.0 / (grid.r + 1j * grid.x)
    yff = ys + 0.5j * grid.b
    shape = (-1,) + (1,) * (V.ndim - 1)
    return yff.reshape(shape) * V[grid.f] - ys.reshape(shape) * V[grid.t]


def branch_loss(grid, V):
    """L = sum_f |I_f|^2 over branches (one value per scenario column of V)."""
    I = branch_currents(grid, V)
    return np.sum(np.abs(I) ** 2, axis=0)


def branch_loss_grad(grid, V):
    """g with dL = Re(sum_k g_k dV_k) (the complex derivative dL/dV, not conjugated).

    dL = sum_f 2 Re(conj(I_f) dI_f) and dI_f = yff dV_f - ys dV_t, so
    g_f += 2 conj(I_f) yff and g_t -= 2 conj(I_f) ys.
    """
    ys = 1.0 / (grid.r + 1j * grid.x)
    yff = ys + 0.5j * grid.b
    I = branch_currents(grid, V)
    shape = (-1,) + (1,) * (V.ndim - 1)
    g = np.zeros_like(V, dtype=np.complex128)
    np.add.at(g, grid.f, 2.0 * np.conj(I) * yff.reshape(shape))
    np.add.at(g, grid.t, -2.0 * np.conj(I) * ys.reshape(shape))
    return g


def loss_state_grad(grid, V):
    """dL/dx for x = [theta over Theta ; |V| over PQ] at one voltage vector V [n].

    An angle step moves V_k by j V_k dtheta_k and a magnitude step by
    (V_k / |V_k|) d|V_k|, so dL/dtheta_k = Re(g_k j V_k) and
    dL/d|V_k| = Re(g_k V_k) / |V_k|.
    """
    theta, pq = nr.index_sets(grid.bus_type)
    g = branch_loss_grad(grid, V)
    d_th = np.real(g * 1j * V)[theta]
    d_vm = (np.real(g * V) / np.abs(V))[pq]
    return np.concatenate([d_th, d_vm])


def dense_adjoint(grid, V):
    """(grad_p [n], grad_q [n]) of the loss w.r.t. the scheduled injections at solution V.

    grad_p is filled on Theta buses (PV and PQ), grad_q on PQ buses, zero elsewhere.
    """
    Y = nr.ybus(grid.n_bus, grid.f, grid.t, grid.r, grid.x, grid.b)
    theta, pq = nr.index_sets(grid.bus_type)
    J = nr.jacobian(Y, V, theta, pq).toarray()
    lam = np.linalg.solve(J.T, loss_state_grad(grid, V))
    gp = np.zeros(grid.n_bus)
    gq = np.zeros(grid.n_bus)
    gp[theta] = lam[:theta.shape[0]]
    gq[pq] = lam[theta.shape[0]:]
    return gp, gq
