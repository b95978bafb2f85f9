"""Pins for the loss gradient and the dense adjoint oracle."""
import numpy as np
import pytest

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


def _reversed(grid):
    """The same grid with every branch's ends swapped (the pi model is symmetric,
    so this changes nothing physical; its from-end currents are the original
    grid's to-end currents)."""
    import dataclasses
    return dataclasses.replace(grid, f=grid.t.copy(), t=grid.f.copy())


@pytest.mark.parametrize("cfg", [tx.TX30, tx.TX2000])
def test_branch_currents_satisfy_kcl_with_the_admittance_matrix(cfg, rng):
    """Pin of the branch currents (pi model, Sec. II-A): for any voltages, the
    current leaving bus i into its branches, from-end currents of the branches
    that start at i plus to-end currents of those that end there, is the bus
    injection (Ybus V)_i of the admittance matrix that the Tellegen pin fixes.
    The to-end currents are the from-end currents of the reversed branches, so
    a charging term counted in full, split unevenly or put on the wrong end
    breaks the balance."""
    grid = tx.make_grid(cfg)
    assert grid.b.max() > 1e-3   # charging present, so the pin sees its split
    B = 3
    V = rng.uniform(0.85, 1.15, (grid.n_bus, B)) * np.exp(1j * rng.uniform(-0.5, 0.5, (grid.n_bus, B)))
    I_f = adjoint.branch_currents(grid, V)
    I_t = adjoint.branch_currents(_reversed(grid), V)
    inj = np.zeros((grid.n_bus, B), dtype=np.complex128)
    np.add.at(inj, grid.f, I_f)
    np.add.at(inj, grid.t, I_t)
    Y = nr.ybus(grid.n_bus, grid.f, grid.t, grid.r, grid.x, grid.b)
    ref = Y @ V
    assert np.abs(inj - ref).max() <= 1e-11 * np.abs(ref).max()
    # complex power: what both ends of every branch draw is what the buses inject
    s_br = V[grid.f] * np.conj(I_f) + V[grid.t] * np.conj(I_t)
    s_bus = np.stack([nr.power(Y, V[:, c]) for c in range(B)], axis=1)
    np.testing.assert_allclose(s_br.sum(axis=0), s_bus.sum(axis=0), rtol=1e-11, atol=1e-11)
    # series current and the half charging at the from end, term by term on one branch
    k = int(np.argmax(grid.b))
    vf, vt = V[grid.f[k], 0], V[grid.t[k], 0]
    z = grid.r[k] + 1j * grid.x[k]
    assert abs(I_f[k, 0] - ((vf - vt) / z + 0.5j * grid.b[k] * vf)) <= 1e-12 * abs(I_f[k, 0])
    # the loss is the sum of the squared from-end current magnitudes
    np.testing.assert_allclose(adjoint.branch_loss(grid, V), np.sum(np.abs(I_f) ** 2, axis=0), rtol=1e-13)


def test_branch_currents_kcl_fails_for_a_planted_charging_error(rng):
    """The KCL pin is sensitive: a branch-current formula that counts the full
    charging at the from end (a plausible slip) violates it."""
    grid = tx.make_grid(tx.TX30)
    V = rng.uniform(0.9, 1.1, grid.n_bus) * np.exp(1j * rng.uniform(-0.3, 0.3, grid.n_bus))

    def wrong(g, v):
        ys = 1.0 / (g.r + 1j * g.x)
        return (ys + 1j * g.b) * v[g.f] - ys * v[g.t]

    inj = np.zeros(grid.n_bus, dtype=np.complex128)
    np.add.at(inj, grid.f, wrong(grid, V))
    np.add.at(inj, grid.t, wrong(_reversed(grid), V))
    Y = nr.ybus(grid.n_bus, grid.f, grid.t, grid.r, grid.x, grid.b)
    assert np.abs(inj - Y @ V).max() > 1e-4
