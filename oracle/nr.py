"""Oracle: Newton-Raphson power flow with a sparse LU Newton step (plain FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed (Sec. II-A):
  * state x = [theta over Theta ; |V| over Q], Theta = PV u PQ, Q = PQ (eq. (1));
  * mismatch F(x) = [P_calc - P over Theta ; Q_calc - Q over Q], with the
    complex bus power S = V * conj(Ybus V) (eq. (2));
  * Newton step J dx = -F, x <- x + dx (eq. (3)), with J the polar Jacobian
    whose blocks are H, N, M, L of eq. (4).

The paper solves the Newton system with preconditioned GMRES; the converged
answer does not depend on the linear solver, so the oracle uses a direct sparse
LU (scipy's SuperLU) for every step.  Convergence: infinity norm of F in per
unit at or below ``tol``, tested before each update, so the iteration count is
the number of updates taken.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import splu

PQ, PV, SLACK = 0, 1, 2


def ybus(n_bus, f, t, r, x, b):
    """Bus admittance matrix of pi-model branches (series r + jx, total charging b).

    Each branch adds y_s + j b/2 to both diagonal entries and -y_s to both
    off-diagonal entries.  Returned as scipy CSR (duplicates summed).
    """
    f = np.asarray(f, dtype=np.int64)
    t = np.asarray(t, dtype=np.int64)
    ys = 1.0 / (np.asarray(r) + 1j * np.asarray(x))
    ysh = 0.5j * np.asarray(b)
    rows = np.concatenate([f, t, f, t])
    cols = np.concatenate([f, t, t, f])
    vals = np.concatenate([ys + ysh, ys + ysh, -ys, -ys])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n_bus, n_bus))


def index_sets(bus_type):
    """(Theta, Q): sorted PV u PQ and sorted PQ bus indices (Sec. II-A)."""
    bt = np.asarray(bus_type)
    theta = np.flatnonzero(bt != SLACK)
    q = np.flatnonzero(bt == PQ)
    return theta, q


def power(Y, V):
    """Complex bus power S = V * conj(Y V) (injection convention)."""
    return V * np.conj(Y @ V)


def mismatch(Y, V, p, q, theta, pq):
    """F = [Re S - P over Theta ; Im S - Q over PQ]  (eq. (2))."""
    S = power(Y, V)
    return np.concatenate([S.real[theta] - p[theta], S.imag[pq] - q[pq]])


def jacobian(Y, V, theta, pq):
    """Polar Jacobian dF/dx as a sparse matrix (blocks H, N / M, L of eq. (4)).

    With I = Y V, a perturbation dV changes the power by
    dS = dV * conj(I) + V * conj(Y dV).  An angle step at bus k moves V_k by
    j V_k dtheta_k, a magnitude step by (V_k / |V_k|) d|V_k|; collecting the
    columns gives
      dS/dtheta = j diag(V) conj(diag(I) - Y diag(V))
      dS/d|V|   = diag(V) conj(Y diag(E)) + conj(diag(I)) diag(E),  E = V / |V|.
    The real parts on Theta rows and the imaginary parts on PQ rows form J.
    """
    I = Y @ V
    DV = sp.diags(V)
    DE = sp.diags(V / np.abs(V))
    DI = sp.diags(I)
    dS_dth = 1j * DV @ (DI - Y @ DV).conj()
    dS_dvm = DV @ (Y @ DE).conj() + DI.conj() @ DE
    dS_dth = dS_dth.tocsr()
    dS_dvm = dS_dvm.tocsr()
    H = dS_dth[theta][:, theta].real
    N = dS_dvm[theta][:, pq].real
    M = dS_dth[pq][:, theta].imag
    L = dS_dvm[pq][:, pq].imag
    return sp.bmat([[H, N], [M, L]], format="csc")


@dataclass
class NRResult:
    V: np.ndarray            # complex128 [n] final bus voltages
    iters: int               # Newton updates taken
    converged: bool
    mismatch: float          # infinity norm of F at the returned V
    history: list            # infinity norm of F before each update (and at the end)


def flat_start(bus_type, vm_set):
    """theta = 0 everywhere, |V| = set-point at PV and slack, 1.0 at PQ buses."""
    vm = np.where(np.asarray(bus_type) == PQ, 1.0, np.asarray(vm_set, dtype=np.float64))
    return vm.astype(np.complex128)


def nr_solve(Y, bus_type, p, q, vm_set, tol=1e-8, max_iter=20, diverge=1e6, V0=None):
    """Newton-Raphson from a flat start (or ``V0``) for one scenario.

    ``p``, ``q``: scheduled injections per bus (generator convention).
    Stops when ||F||_inf <= tol (converged), when ``max_iter`` updates were
    taken, or when F is non-finite or exceeds ``diverge`` (not converged).
    """
    theta, pq = index_sets(bus_type)
    nth = theta.shape[0]
    V = flat_start(bus_type, vm_set) if V0 is None else np.array(V0, dtype=np.complex128)
    ang = np.angle(V)
    vm = np.abs(V)
    hist = []
    for k in range(max_iter + 1):
        F = mismatch(Y, V, p, q, theta, pq)
        nf = float(np.max(np.abs(F))) if F.size else 0.0
        hist.append(nf)
        if not np.isfinite(nf) or nf > diverge:
            return NRResult(V, k, False, nf, hist)
        if nf <= tol:
            return NRResult(V, k, True, nf, hist)
        if k == max_iter:
            break
        J = jacobian(Y, V, theta, pq)
        dx = splu(J).solve(-F)
        ang[theta] += dx[:nth]
        vm[pq] += dx[nth:]
        V = vm * np.exp(1j * ang)
    return NRResult(V, max_iter, False, hist[-1], hist)


def nr_solve_batch(grid, batch, tol=1e-8, max_iter=20, columns=None):
    """Solve the scenarios of a ``workloads.transmission`` batch one by one.

    Returns (V [nb, n] complex, iters [nb], converged [nb], mismatch [nb]) for
    the requested scenarios ``columns`` (default: all).
    """
    Y = ybus(grid.n_bus, grid.f, grid.t, grid.r, grid.x, grid.b)
    cols = np.arange(batch.batch) if columns is None else np.asarray(columns)
    V = np.zeros((cols.shape[0], grid.n_bus), dtype=np.complex128)
    it = np.zeros(cols.shape[0], dtype=np.int32)
    ok = np.zeros(cols.shape[0], dtype=bool)
    mm = np.zeros(cols.shape[0])
    for j, c in enumerate(cols):
        res = nr_solve(Y, grid.bus_type, batch.p_inj[c], batch.q_inj[c], batch.vm_set[c],
                       tol=tol, max_iter=max_iter)
        V[j] = res.V
        it[j] = res.iters
        ok[j] = res.converged
        mm[j] = res.mismatch
    return V, it, ok, mm
