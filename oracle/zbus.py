"""Oracle: three-phase Z-bus fixed-point power flow on a radial feeder (plain FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed (Sec. II-B, eq. (10)):
  * the three-phase bus admittance matrix over phase nodes, split into slack
    phases S (the substation) and the rest N;
  * the reduced bus-impedance matrix Z = inv(Y_NN) and the no-load voltage
    v0 = -Z Y_NS v_S;
  * the current-injection map i(v): wye loads inject -conj(S / v); delta loads
    draw branch currents conj(S_ab / v_ab) etc. from line-to-line voltages,
    mapped back to phase injections;
  * the fixed point v <- Z i(v) + v0 from v = v0, run literally (eq. (10)).

The paper stops when the change in the sum of voltage magnitudes is small or
at an iteration cap.  The oracle iterates to a much tighter voltage-change
criterion (max |v_{k+1} - v_k| <= 1e-13) and reports, for each scenario, the
per-node power mismatch v * conj(r) with r = i(v) - (Y_NN v + Y_NS v_S), and
the paper's sum-of-magnitudes change of the last step.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SLACK_NODES = np.array([0, 1, 2])


def ybus3(feeder):
    """Dense three-phase Ybus over all phase nodes (node = 3*bus + phase).

    Each segment with 3x3 series impedance z adds y = inv(z) to the two
    diagonal 3x3 blocks and -y to the two off-diagonal blocks (no shunts).
    """
    n = feeder.n_node
    Y = np.zeros((n, n), dtype=np.complex128)
    for s in range(feeder.n_seg):
        y = np.linalg.inv(feeder.z_seg[s])
        a = 3 * int(feeder.seg_from[s])
        c = 3 * int(feeder.seg_to[s])
        Y[a:a + 3, a:a + 3] += y
        Y[c:c + 3, c:c + 3] += y
        Y[a:a + 3, c:c + 3] -= y
        Y[c:c + 3, a:a + 3] -= y
    return Y


def split(feeder):
    """(Y_NN, Y_NS, non-slack node indices) with the substation phases as S."""
    Y = ybus3(feeder)
    N = np.setdiff1d(np.arange(feeder.n_node), SLACK_NODES)
    return Y[np.ix_(N, N)], Y[np.ix_(N, SLACK_NODES)], N


def zbus(feeder):
    """(Z, v0, N): reduced bus-impedance matrix, no-load voltage, node list."""
    YNN, YNS, N = split(feeder)
    Z = np.linalg.inv(YNN)
    v0 = -Z @ (YNS @ feeder.v_slack)
    return Z, v0, N


def injection(v, s_wye, s_delta, delta_nodes):
    """Load current injections i(v) over the phase nodes ``v`` indexes.

    ``v``, ``s_wye``, ``s_delta``: [n, B] complex over the same node list.
    ``delta_nodes``: [n_delta, 3] rows (a, b, c) into that node list, with the
    ab, bc, ca branch loads stored at rows a, b, c of ``s_delta``.
    """
    i = -np.conj(s_wye / v)
    if len(delta_nodes):
        a, b, c = delta_nodes[:, 0], delta_nodes[:, 1], delta_nodes[:, 2]
        v_ab = v[a] - v[b]
        v_bc = v[b] - v[c]
        v_ca = v[c] - v[a]
        i_ab = np.conj(s_delta[a] / v_ab)
        i_bc = np.conj(s_delta[b] / v_bc)
        i_ca = np.conj(s_delta[c] / v_ca)
        i[a] += -(i_ab - i_ca)
        i[b] += -(i_bc - i_ab)
        i[c] += -(i_ca - i_bc)
    return i


def _nonslack_delta(feeder, N):
    pos = -np.ones(feeder.n_node, dtype=np.int64)
    pos[N] = np.arange(N.shape[0])
    d = feeder.delta_nodes
    return pos[d] if len(d) else np.zeros((0, 3), dtype=np.int64)


@dataclass
class ZbusResult:
    v: np.ndarray              # complex128 [B, n_node] all phase nodes incl. the slack
    iters: np.ndarray          # int32 [B] fixed-point updates until the stop rule
    converged: np.ndarray      # bool [B]: voltage change reached tol_v
    mismatch: np.ndarray       # float64 [B] max |v * conj(r)| over non-slack nodes
    sum_abs_change: np.ndarray # float64 [B] |sum |v_k+1| - sum |v_k|| of the last step


def residual(feeder, v_all, s_wye, s_delta):
    """r = i(v) - (Y_NN v_N + Y_NS v_S) over the non-slack nodes, and the mismatch v * conj(r).

    Arguments and results are node-major ([n_node, B] in, [nN, B] out)."""
    YNN, YNS, N = split(feeder)
    dN = _nonslack_delta(feeder, N)
    vN = v_all[N]
    r = injection(vN, s_wye[N], s_delta[N], dN) - (YNN @ vN + (YNS @ v_all[SLACK_NODES]))
    return r, vN * np.conj(r)


def zbus_solve(feeder, batch, tol_v=1e-13, max_iter=200, setup=None):
    """Run v <- Z i(v) + v0 from v0 for every scenario of the batch (eq. (10)).

    ``setup`` may pass a precomputed ``zbus(feeder)`` result."""
    Z, v0, N = zbus(feeder) if setup is None else setup
    dN = _nonslack_delta(feeder, N)
    sw = batch.s_wye.T[N]
    sd = batch.s_delta.T[N]
    B = batch.batch
    v = np.repeat(v0[:, None], B, axis=1)
    iters = np.full(B, max_iter, dtype=np.int32)
    done = np.zeros(B, dtype=bool)
    last_sum_change = np.zeros(B)
    for k in range(1, max_iter + 1):
        v_new = Z @ injection(v, sw, sd, dN) + v0[:, None]
        dv = np.max(np.abs(v_new - v), axis=0)
        sum_change = np.abs(np.abs(v_new).sum(axis=0) - np.abs(v).sum(axis=0))
        upd = ~done
        v[:, upd] = v_new[:, upd]
        last_sum_change[upd] = sum_change[upd]
        newly = upd & (dv <= tol_v)
        iters[newly] = k
        done |= newly
        if done.all():
            break
    v_all = np.zeros((feeder.n_node, B), dtype=np.complex128)
    v_all[SLACK_NODES] = feeder.v_slack[:, None]
    v_all[N] = v
    _, dS = residual(feeder, v_all, batch.s_wye.T, batch.s_delta.T)
    mm = np.max(np.abs(dS), axis=0)
    return ZbusResult(v=v_all.T.copy(), iters=iters, converged=done, mismatch=mm,
                      sum_abs_change=last_sum_change)
