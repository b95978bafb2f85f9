"""Pins for the three-phase Z-bus oracle (Sec. II-B, eq. (10))."""
import numpy as np
import pytest

from oracle import zbus
from workloads import feeder as fdm


@pytest.fixture(scope="module")
def small_feeder():
    cfg = fdm.FeederConfig("feeder40", n_bus=40, max_depth=25, batch=8, seed=41)
    fd = fdm.make_feeder(cfg)
    return fd, fdm.make_batch(fd, cfg)


def _path(fd, bus):
    segs = []
    while bus != 0:
        segs.append(bus - 1)           # segment k feeds bus k + 1
        bus = int(fd.parent[bus])
    return set(segs)


def test_radial_zbus_closed_form(small_feeder):
    """Block (i, j) of Z is the sum of segment impedances shared by the root paths of i and j."""
    fd, _ = small_feeder
    Z, v0, N = zbus.zbus(fd)
    assert np.all(fd.seg_to == np.arange(1, fd.n_bus))
    Zc = np.zeros((fd.n_node, fd.n_node), dtype=np.complex128)
    paths = [_path(fd, i) for i in range(fd.n_bus)]
    for i in range(1, fd.n_bus):
        for j in range(1, fd.n_bus):
            for s in paths[i] & paths[j]:
                Zc[3 * i:3 * i + 3, 3 * j:3 * j + 3] += fd.z_seg[s]
    Zc = Zc[np.ix_(N, N)]
    assert np.max(np.abs(Z - Zc)) <= 1e-12 * np.max(np.abs(Zc))
    v_rep = np.tile(fd.v_slack, fd.n_bus - 1)
    assert np.max(np.abs(v0 - v_rep)) <= 1e-12


def test_zero_load_gives_no_load_voltage(small_feeder):
    fd, _ = small_feeder
    res = zbus.zbus_solve(fd, fdm.zero_load(fd, 2))
    assert res.converged.all() and np.all(res.iters == 1)
    v_rep = np.tile(fd.v_slack, fd.n_bus)
    assert np.max(np.abs(res.v - v_rep[None, :])) <= 1e-13
    # Y v cancels entries of size max|Y| ~ 1e3 pu: rounding leaves ~1e-12
    assert res.mismatch.max() <= 1e-11


def test_power_balance_from_segment_data(small_feeder):
    """Substation injection = specified wye + delta loads + series losses, from segment currents."""
    fd, batch = small_feeder
    res = zbus.zbus_solve(fd, batch)
    assert res.converged.all()
    for b in range(batch.batch):
        v = res.v[b].reshape(fd.n_bus, 3)
        s_slack = 0.0
        losses = 0.0
        for s in range(fd.n_seg):
            p, c = int(fd.seg_from[s]), int(fd.seg_to[s])
            i_seg = np.linalg.solve(fd.z_seg[s], v[p] - v[c])
            losses += np.sum(np.conj(i_seg) * (fd.z_seg[s] @ i_seg))
            if p == 0:
                s_slack += np.sum(v[0] * np.conj(i_seg))
        loads = batch.s_wye[b].sum() + batch.s_delta[b].sum()
        assert abs(s_slack - (loads + losses)) <= 1e-9 * abs(s_slack)


def _closed_form_phase_a(z1, s):
    r, x, p, q = z1.real, z1.imag, s.real, s.imag
    a = r * p + x * q
    c = x * p - r * q
    bq = 2 * a - 1.0
    u = (-bq + np.sqrt(bq * bq - 4 * (a * a + c * c))) / 2
    return np.sqrt(u) * np.exp(-1j * np.arctan2(c, u + a))


@pytest.mark.parametrize("kind", [1, 2])
def test_balanced_segment_reduces_to_two_bus(kind):
    """Balanced load on one coupled segment: phase a follows the single-phase closed form
    with the positive-sequence impedance z_self - z_mutual."""
    z_self = 0.03 + 0.06j
    kappa = 0.4
    s = 2.0 + 0.7j
    fd, batch = fdm.single_segment(z_self, kappa, kind, s)
    res = zbus.zbus_solve(fd, batch)
    assert res.converged.all()
    va = _closed_form_phase_a(z_self * (1 - kappa), s)
    a = np.exp(-2j * np.pi / 3)
    expect = np.array([va, va * a, va * a * a])
    assert np.max(np.abs(res.v[0, 3:6] - expect)) <= 1e-12


def test_delta_and_wye_injection_conserve_power(rng):
    """Power drawn through the injection map equals the specified loads at any voltage."""
    n_bus = 5
    v = (rng.uniform(0.9, 1.1, (3 * n_bus, 4)) *
         np.exp(1j * (np.tile(np.array([0, -2, 2]) * np.pi / 3, n_bus)[:, None] + rng.uniform(-0.1, 0.1, (3 * n_bus, 4)))))
    sw = np.zeros((3 * n_bus, 4), dtype=np.complex128)
    sd = np.zeros_like(sw)
    sw[0:3] = rng.uniform(0, 1, (3, 4)) + 1j * rng.uniform(0, 1, (3, 4))
    sd[6:9] = rng.uniform(0, 1, (3, 4)) + 1j * rng.uniform(0, 1, (3, 4))
    delta = np.array([[6, 7, 8]])
    i = zbus.injection(v, sw, sd, delta)
    drawn = -(v * np.conj(i))
    np.testing.assert_allclose(drawn[0:3], sw[0:3], rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(drawn[6:9].sum(axis=0), sd[6:9].sum(axis=0), rtol=1e-13)
    np.testing.assert_allclose(i[6:9].sum(axis=0), 0, atol=1e-13)   # no neutral current from delta


def test_paper_stop_quantity_is_small(small_feeder):
    fd, batch = small_feeder
    res = zbus.zbus_solve(fd, batch)
    assert res.sum_abs_change.max() <= 1e-10
    assert res.mismatch.max() <= 1e-10
