"""Seeded generators: determinism, structure and feasibility in the oracle."""
import numpy as np
import pytest

from oracle import nr, zbus
from workloads import feeder as fdm
from workloads import serving, transmission as tx


def _same(a, b):
    for k, v in a.__dict__.items():
        w = b.__dict__[k]
        if isinstance(v, np.ndarray):
            np.testing.assert_array_equal(v, w)
        else:
            assert v == w


@pytest.mark.parametrize("cfg", [tx.TX30, tx.TX2000])
def test_grid_is_deterministic_and_well_formed(cfg):
    g1, g2 = tx.make_grid(cfg), tx.make_grid(cfg)
    _same(g1, g2)
    n = cfg.n_bus
    assert g1.n_branch == cfg.n_branch
    assert np.sum(g1.bus_type == tx.SLACK) == 1 and g1.n_pv == cfg.n_pv
    assert g1.n_pq == n - cfg.n_pv - 1
    assert np.all(g1.f != g1.t)
    keys = set(zip(np.minimum(g1.f, g1.t).tolist(), np.maximum(g1.f, g1.t).tolist()))
    assert len(keys) == g1.n_branch
    deg = np.bincount(np.concatenate([g1.f, g1.t]), minlength=n)
    assert deg.min() >= 1 and abs(deg.mean() - 2 * cfg.n_branch / n) < 1e-12
    # connected
    seen = {g1.slack}
    stack = [g1.slack]
    adj = tx._adjacency(n, g1.f, g1.t)
    while stack:
        u = stack.pop()
        for w in adj[u]:
            if w not in seen:
                seen.add(w)
                stack.append(w)
    assert len(seen) == n
    assert np.all((g1.x / g1.r >= 2) & (g1.x / g1.r <= 6))
    pq = g1.bus_type == tx.PQ
    np.testing.assert_allclose(g1.q_load[pq], 0.3 * g1.p_load[pq])
    assert np.all(g1.p_load[~pq] == 0)


def test_batches_are_deterministic():
    g = tx.make_grid(tx.TX30)
    _same(tx.make_batch(g, tx.TX30), tx.make_batch(g, tx.TX30))
    b = tx.make_batch(g, tx.TX30)
    pq = g.bus_type == tx.PQ
    ratio = b.p_inj[:, pq] / (-g.p_load[pq][None, :])
    np.testing.assert_allclose(ratio, ratio[:, 0:1].repeat(ratio.shape[1], 1))   # one factor per scenario


def test_tx30_all_scenarios_converge_in_oracle():
    g = tx.make_grid(tx.TX30)
    b = tx.make_batch(g, tx.TX30)
    V, it, ok, mm = nr.nr_solve_batch(g, b)
    assert ok.all() and mm.max() <= 1e-8 and np.abs(V).min() > 0.7


@pytest.mark.slow
def test_tx2000_sample_converges_in_oracle():
    g = tx.make_grid(tx.TX2000)
    b = tx.make_batch(g, tx.TX2000)
    V, it, ok, mm = nr.nr_solve_batch(g, b, columns=np.arange(0, 1024, 128))
    assert ok.all() and np.abs(V).min() > 0.7


def test_feeder_structure():
    cfg = fdm.FEEDER300
    f1, f2 = fdm.make_feeder(cfg), fdm.make_feeder(cfg)
    _same(f1, f2)
    assert f1.n_node == 900 and f1.n_seg == 299
    assert f1.depth.max() <= cfg.max_depth
    assert np.sum(f1.load_kind == 1) == 179 and np.sum(f1.load_kind == 2) == 120
    assert f1.load_kind[0] == 0
    assert f1.delta_nodes.shape == (120, 3)
    # lagging 0.95 power factor
    s = f1.s_base_wye[f1.s_base_wye != 0]
    np.testing.assert_allclose(s.real / np.abs(s), 0.95)


def test_feeder_sample_converges_in_oracle():
    cfg = fdm.FEEDER300
    fd = fdm.make_feeder(cfg)
    res = zbus.zbus_solve(fd, fdm.make_batch(fd, cfg, batch=16))
    assert res.converged.all() and res.mismatch.max() <= 1e-10
    assert np.abs(res.v).min() > 0.85


def test_serving_trace():
    tr = serving.make_trace(n_requests=5000)
    assert tr == serving.make_trace(n_requests=5000)
    k = np.array([r.n_scen for r in tr])
    assert k.min() >= 1 and k.max() <= 512
    t = np.array([r.t_arrive for r in tr])
    assert np.all(np.diff(t) >= 0)
    rate = (len(tr) - 1) / t[-1]
    assert abs(rate - 2000) / 2000 < 0.05
    assert set(r.network for r in tr) == {0, 1, 2}


def test_outage_batches_keep_the_grid_connected():
    import numpy as np
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    from workloads import transmission as tx

    grid = tx.make_grid(tx.TX30)
    for n_out in (0, 1, 3):
        on = tx.make_outages(grid, 20, n_out=n_out, seed=11)
        assert on.dtype == np.uint8 and on.shape == (20, grid.f.shape[0])
        assert ((on == 0).sum(axis=1) == n_out).all()
        for s in range(20):
            m = on[s].astype(bool)
            g = coo_matrix((np.ones(int(m.sum())), (grid.f[m], grid.t[m])), shape=(grid.n_bus, grid.n_bus))
            assert connected_components(g, directed=False)[0] == 1
    np.testing.assert_array_equal(tx.make_outages(grid, 5, 2, seed=1), tx.make_outages(grid, 5, 2, seed=1))
