"""Pins for the loss gradient and the dense adjoint oracle."""
import numpy as np

from oracle import adjoint, nr
from workloads import transmission as tx
from tests.test_oracle_nr import two_bus_closed_form


def test_loss_gradient_matches_finite_differences(rng):
    grid = tx.make_grid(tx.TX30)
    V = rng.uniform(0.9, 1.1, grid.n_bus) * np.exp(1j * rng.uniform(-0.2, 0.2, grid.n_bus))
    g = adjoint.branch_loss_grad(grid, V)
    h = 1e-6
    for k in range(0, grid.n_bus, 3):
        for d in (1.0, 1j):
            e = np.zeros(grid.n_bus, dtype=np.complex128)
            e[k] = h * d
            fd = (adjoint.branch_loss(grid, V + e) - adjoint.branch_loss(grid, V - e)) / (2 * h)
            assert abs(fd - np.real(g[k] * d)) <= 1e-7 * max(1.0, abs(g[k]))


def test_dense_adjoint_matches_central_differences():
    grid = tx.make_grid(tx.TX30)
    batch = tx.make_batch(grid, tx.TX30)
    Y = nr.ybus(grid.n_bus, grid.f, grid.t, grid.r, grid.x, grid.b)
    col = 3
    p0, q0, vs = batch.p_inj[col], batch.q_inj[col], batch.vm_set[col]
    res = nr.nr_solve(Y, grid.bus_type, p0, q0, vs, tol=1e-13)
    gp, gq = adjoint.dense_adjoint(grid, res.V)
    h = 1e-6
    theta, pq = nr.index_sets(grid.bus_type)
    scale = max(np.abs(gp).max(), np.abs(gq).max())

    def L(p, q):
        r = nr.nr_solve(Y, grid.bus_type, p, q, vs, tol=1e-13, V0=res.V)
        assert r.converged
        return adjoint.branch_loss(grid, r.V)

    for k in theta[::4]:
        e = np.zeros(grid.n_bus)
        e[k] = h
        fd = (L(p0 + e, q0) - L(p0 - e, q0)) / (2 * h)
        assert abs(fd - gp[k]) <= 1e-6 * scale
    for k in pq[::4]:
        e = np.zeros(grid.n_bus)
        e[k] = h
        fd = (L(p0, q0 + e) - L(p0, q0 - e)) / (2 * h)
        assert abs(fd - gq[k]) <= 1e-6 * scale
    assert gp[grid.slack] == 0 and np.all(gq[grid.bus_type != tx.PQ] == 0)


def test_two_bus_adjoint_matches_closed_form():
    """dL/dP of the 2-bus case from finite differences of the closed-form voltage."""
    r, x, P, Q = 0.03, 0.12, 0.8, 0.25
    grid, batch = tx.two_bus(r, x, P, Q)
    Y = nr.ybus(grid.n_bus, grid.f, grid.t, grid.r, grid.x, grid.b)
    res = nr.nr_solve(Y, grid.bus_type, batch.p_inj[0], batch.q_inj[0], batch.vm_set[0],
                      tol=1e-14)
    gp, gq = adjoint.dense_adjoint(grid, res.V)

    def L(Pl, Ql):
        vm, th = two_bus_closed_form(r, x, Pl, Ql)
        return abs((1.0 - vm * np.exp(1j * th)) / (r + 1j * x)) ** 2

    h = 1e-6
    # injections are minus the consumption
    dLdp = -(L(P + h, Q) - L(P - h, Q)) / (2 * h)
    dLdq = -(L(P, Q + h) - L(P, Q - h)) / (2 * h)
    assert abs(gp[1] - dLdp) <= 1e-8
    assert abs(gq[1] - dLdq) <= 1e-8
