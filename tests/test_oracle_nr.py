"""Pins for the Newton-Raphson oracle (Sec. II-A, eqs. (1)-(4)).

Each test checks the oracle against something other than itself: a closed
form, an exact special case, an identity computed from branch data, finite
differences, or an independent nonlinear solver.
"""
import numpy as np
import pytest
from scipy.optimize import fsolve

from oracle import nr
from workloads import transmission as tx


def two_bus_closed_form(r, x, p, q, v1=1.0):
    """|V2| and angle of V2 for a slack at v1∠0 feeding load p + jq over r + jx.

    With a = rp + xq and c = xp - rq, u = |V2|^2 solves
    u^2 + (2a - v1^2) u + a^2 + c^2 = 0 (high-voltage root) and
    theta2 = -atan2(c, u + a).
    """
    a = r * p + x * q
    c = x * p - r * q
    bq = 2 * a - v1 ** 2
    u = (-bq + np.sqrt(bq * bq - 4 * (a * a + c * c))) / 2
    return np.sqrt(u), -np.arctan2(c, u + a)


@pytest.mark.parametrize("r,x,p,q", [(0.02, 0.1, 0.5, 0.2), (0.05, 0.05, 1.2, -0.3),
                                     (0.01, 0.3, 0.8, 0.4), (0.1, 0.2, 0.0, 0.5),
                                     (0.03, 0.12, -0.4, 0.1)])
def test_two_bus_closed_form(r, x, p, q):
    grid, batch = tx.two_bus(r, x, p, q)
    Y = nr.ybus(grid.n_bus, grid.f, grid.t, grid.r, grid.x, grid.b)
    res = nr.nr_solve(Y, grid.bus_type, batch.p_inj[0], batch.q_inj[0], batch.vm_set[0],
                      tol=1e-13)
    vm, th = two_bus_closed_form(r, x, p, q)
    assert res.converged
    assert abs(np.abs(res.V[1]) - vm) <= 1e-12
    assert abs(np.angle(res.V[1]) - th) <= 1e-12
    assert res.V[0] == 1.0


def test_zero_load_flat_start_is_solution():
    grid = tx.make_grid(tx.TX30)
    grid.b = np.zeros_like(grid.b)
    Y = nr.ybus(grid.n_bus, grid.f, grid.t, grid.r, grid.x, grid.b)
    batch = tx.zero_load(grid)
    res = nr.nr_solve(Y, grid.bus_type, batch.p_inj[0], batch.q_inj[0], batch.vm_set[0])
    assert res.converged and res.iters == 0
    assert res.mismatch <= 1e-14
    np.testing.assert_array_equal(res.V, np.ones(grid.n_bus))


def test_power_balance_from_branch_data(rng):
    """Sum of bus powers equals series losses minus charging vars, for any V (Tellegen)."""
    grid = tx.make_grid(tx.TX30)
    Y = nr.ybus(grid.n_bus, grid.f, grid.t, grid.r, grid.x, grid.b)
    for _ in range(3):
        V = rng.uniform(0.9, 1.1, grid.n_bus) * np.exp(1j * rng.uniform(-0.3, 0.3, grid.n_bus))
        total = nr.power(Y, V).sum()
        zs = grid.r + 1j * grid.x
        Is = (V[grid.f] - V[grid.t]) / zs
        branch = np.sum(np.abs(Is) ** 2 * zs - 0.5j * grid.b * (np.abs(V[grid.f]) ** 2 + np.abs(V[grid.t]) ** 2))
        assert abs(total - branch) <= 1e-12 * max(1.0, abs(branch))


def test_jacobian_matches_central_differences(rng):
    grid = tx.make_grid(tx.TX30)
    Y = nr.ybus(grid.n_bus, grid.f, grid.t, grid.r, grid.x, grid.b)
    theta, pq = nr.index_sets(grid.bus_type)
    batch = tx.make_batch(grid, tx.TX30)
    p, q = batch.p_inj[0], batch.q_inj[0]
    ang = rng.uniform(-0.2, 0.2, grid.n_bus)
    vm = rng.uniform(0.95, 1.05, grid.n_bus)
    x0 = np.concatenate([ang[theta], vm[pq]])

    def F(x):
        a = ang.copy()
        m = vm.copy()
        a[theta] = x[:theta.shape[0]]
        m[pq] = x[theta.shape[0]:]
        return nr.mismatch(Y, m * np.exp(1j * a), p, q, theta, pq)

    J = nr.jacobian(Y, vm * np.exp(1j * ang), theta, pq).toarray()
    h = 1e-6
    Jfd = np.empty_like(J)
    for k in range(x0.shape[0]):
        e = np.zeros_like(x0)
        e[k] = h
        Jfd[:, k] = (F(x0 + e) - F(x0 - e)) / (2 * h)
    assert np.max(np.abs(J - Jfd)) <= 1e-7 * np.max(np.abs(J))


def test_nr_matches_independent_solver():
    """The LU-Newton solution agrees with MINPACK's hybrid method on the same F."""
    grid = tx.make_grid(tx.TX30)
    batch = tx.make_batch(grid, tx.TX30)
    Y = nr.ybus(grid.n_bus, grid.f, grid.t, grid.r, grid.x, grid.b)
    theta, pq = nr.index_sets(grid.bus_type)
    for col in (0, 17, 63):
        p, q, vs = batch.p_inj[col], batch.q_inj[col], batch.vm_set[col]
        res = nr.nr_solve(Y, grid.bus_type, p, q, vs, tol=1e-12)
        base_vm = np.where(grid.bus_type == tx.PQ, 1.0, vs)

        def F(x):
            a = np.zeros(grid.n_bus)
            m = base_vm.copy()
            a[theta] = x[:theta.shape[0]]
            m[pq] = x[theta.shape[0]:]
            return nr.mismatch(Y, m * np.exp(1j * a), p, q, theta, pq)

        x0 = np.concatenate([np.zeros(theta.shape[0]), np.ones(pq.shape[0])])
        xs = fsolve(F, x0, xtol=1e-14)
        assert np.max(np.abs(F(xs))) < 1e-10
        assert res.converged
        np.testing.assert_allclose(np.angle(res.V[theta]), xs[:theta.shape[0]], atol=1e-9)
        np.testing.assert_allclose(np.abs(res.V[pq]), xs[theta.shape[0]:], atol=1e-9)


def test_quadratic_convergence():
    """Newton with the exact Jacobian: each error is about the square of the previous one."""
    grid = tx.make_grid(tx.TX30)
    batch = tx.make_batch(grid, tx.TX30)
    Y = nr.ybus(grid.n_bus, grid.f, grid.t, grid.r, grid.x, grid.b)
    res = nr.nr_solve(Y, grid.bus_type, batch.p_inj[5], batch.q_inj[5], batch.vm_set[5],
                      tol=1e-14)
    h = np.asarray(res.history)
    h = h[h > 1e-13]
    ratios = np.log(h[2:]) / np.log(h[1:-1])
    assert ratios[-1] > 1.6


def test_index_sets_and_flat_start():
    grid = tx.make_grid(tx.TX30)
    theta, pq = nr.index_sets(grid.bus_type)
    assert theta.shape[0] == 29 and pq.shape[0] == 24
    assert grid.slack not in theta
    v = nr.flat_start(grid.bus_type, grid.vm_set)
    assert np.all(np.angle(v) == 0)
    assert np.all(np.abs(v)[pq] == 1.0)
    pv = np.flatnonzero(grid.bus_type == tx.PV)
    np.testing.assert_array_equal(np.abs(v)[pv], grid.vm_set[pv])


def test_nonconvergence_is_reported():
    grid = tx.make_grid(tx.TX30)
    batch = tx.make_batch(grid, tx.TX30)
    Y = nr.ybus(grid.n_bus, grid.f, grid.t, grid.r, grid.x, grid.b)
    res = nr.nr_solve(Y, grid.bus_type, 50 * batch.p_inj[0], 50 * batch.q_inj[0],
                      batch.vm_set[0])
    assert not res.converged
    res1 = nr.nr_solve(Y, grid.bus_type, batch.p_inj[0], batch.q_inj[0], batch.vm_set[0],
                       max_iter=1)
    assert not res1.converged and res1.iters == 1
