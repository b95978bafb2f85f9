"""Newton-Raphson on the GPU against the CPU oracle (parity: 1e-6 pu in |V|,
1e-6 rad in angle, converged mismatch <= 1e-8 pu)."""
import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import nr as onr
from tests.gpu_common import HV_FLOOR_TX, angle_err, assert_high_voltage, say, spread_cols, to_dev
from workloads import transmission as tx

pytestmark = pytest.mark.gpu

TOL_V = 1e-6
TOL_A = 1e-6


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2605_14103_amd import pf
    assert torch.cuda.is_available()
    c = pf.Context(0)
    yield c
    c.close()


def _solve(net, batch, **opts):
    p = to_dev(batch.p_inj)
    q = to_dev(batch.q_inj)
    vm = to_dev(batch.vm_set)
    res = net.solve(p, q, vm, **opts)
    import torch
    torch.cuda.synchronize()
    return res


def _check_against_oracle(grid, batch, res, cols, precision):
    V, it, ok, mm = onr.nr_solve_batch(grid, batch, columns=cols)
    assert ok.all()
    v = res.v.cpu().numpy()[cols]
    da, dm = angle_err(v, V)
    conv = res.converged.cpu().numpy()[cols]
    mis = res.mismatch.cpu().numpy()[cols]
    say(f"{grid.name} {precision}: max angle err {da:.2e} rad, max |V| err {dm:.2e} pu, "
        f"mismatch max {mis.max():.2e}, newton {res.newton_iters.cpu().numpy()[cols].tolist()[:8]}, "
        f"gmres {res.gmres_iters.cpu().numpy()[cols].tolist()[:8]}")
    assert conv.all()
    assert mis.max() <= 1e-8
    assert da <= TOL_A and dm <= TOL_V


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tx30_full_batch(ctx, precision):
    from paper_2605_14103_amd import pf
    say("tx30", precision)
    grid = tx.make_grid(tx.TX30)
    batch = tx.make_batch(grid, tx.TX30)
    net = pf.TxNetwork.from_grid(ctx, grid)
    res = _solve(net, batch, precision=pf.precision(precision))
    assert_high_voltage(res.v.cpu().numpy(), HV_FLOOR_TX, f"tx30 {precision}")
    _check_against_oracle(grid, batch, res, np.arange(batch.batch), precision)
    net.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tx2000_full_batch_sampled(ctx, precision):
    """The 2000-bus grid at its full batch of 1024; sampled scenarios against the oracle."""
    from paper_2605_14103_amd import pf
    say("tx2000", precision)
    grid = tx.make_grid(tx.TX2000)
    batch = tx.make_batch(grid, tx.TX2000)
    net = pf.TxNetwork.from_grid(ctx, grid)
    say("tx2000 factor info", net.info)
    res = _solve(net, batch, precision=pf.precision(precision))
    assert res.converged.cpu().numpy().all()
    assert res.mismatch.cpu().numpy().max() <= 1e-8
    assert_high_voltage(res.v.cpu().numpy(), HV_FLOOR_TX, f"tx2000 {precision}")
    _check_against_oracle(grid, batch, res, spread_cols(batch.batch, 32), precision)
    net.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tx2000_full_occupancy_repeatable(ctx, precision):
    """Batches of 512 and 1024 (two and four workgroups per CU) solved twice: every
    scenario converged and both runs bit-identical, and each scenario of the
    1024 batch bit-identical to the same scenario solved in a batch of 256.  A
    workspace written with 16-byte stores once gave a few percent of the
    scenarios beyond the first workgroup per CU wrong values, different ones
    from run to run; this is the check that caught it."""
    from paper_2605_14103_amd import pf
    grid = tx.make_grid(tx.TX2000)
    batch = tx.make_batch(grid, tx.TX2000)
    net = pf.TxNetwork.from_grid(ctx, grid)
    o = dict(precision=pf.precision(precision))
    p, q, vm = to_dev(batch.p_inj), to_dev(batch.q_inj), to_dev(batch.vm_set)
    import torch
    for B in (512, 1024):
        a = net.solve(p[:B], q[:B], vm[:B], **o)
        torch.cuda.synchronize()
        va = a.v.cpu().numpy()
        b = net.solve(p[:B], q[:B], vm[:B], **o)
        torch.cuda.synchronize()
        say(f"tx2000 {precision} batch {B}: converged {int(a.converged.sum())}, "
            f"max mismatch {float(a.mismatch.max()):.2e}")
        assert a.converged.cpu().numpy().all() and b.converged.cpu().numpy().all()
        np.testing.assert_array_equal(va, b.v.cpu().numpy())
        np.testing.assert_array_equal(a.gmres_iters.cpu().numpy(), b.gmres_iters.cpu().numpy())
    # the last quarter of the 1024 batch (fourth workgroup per CU) against the
    # same scenarios alone in a batch of 256 (one workgroup per CU)
    c = net.solve(p[768:], q[768:], vm[768:], **o)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(va[768:], c.v.cpu().numpy())
    net.close()


@pytest.mark.parametrize("direct", [0, 1])
def test_two_bus_closed_form(ctx, direct):
    from paper_2605_14103_amd import pf
    from tests.test_oracle_nr import two_bus_closed_form
    grid, batch = tx.two_bus(0.03, 0.12, 0.8, 0.25, batch=3)
    net = pf.TxNetwork.from_grid(ctx, grid)
    res = _solve(net, batch, tol=1e-12, nr_direct=direct)
    vm, th = two_bus_closed_form(0.03, 0.12, 0.8, 0.25)
    v = res.v.cpu().numpy()
    assert res.converged.cpu().numpy().all()
    np.testing.assert_allclose(np.abs(v[:, 1]), vm, atol=1e-12)
    np.testing.assert_allclose(np.angle(v[:, 1]), th, atol=1e-12)
    net.close()


@pytest.mark.parametrize("direct", [0, 1])
def test_zero_load_takes_no_iteration(ctx, direct):
    from paper_2605_14103_amd import pf
    grid = tx.make_grid(tx.TX30)
    grid.b = np.zeros_like(grid.b)
    net = pf.TxNetwork.from_grid(ctx, grid)
    res = _solve(net, tx.zero_load(grid, batch=2), nr_direct=direct)
    assert res.converged.cpu().numpy().all()
    assert (res.newton_iters.cpu().numpy() == 0).all()
    np.testing.assert_array_equal(res.v.cpu().numpy(), np.ones((2, grid.n_bus)))
    net.close()


def test_edge_cases_and_isolation(ctx):
    """Empty batch, padded rows, an infeasible and a NaN scenario next to good ones,
    an iteration cap of one; the good scenarios must be bitwise unaffected."""
    import torch
    from paper_2605_14103_amd import pf
    grid = tx.make_grid(tx.TX30)
    batch = tx.make_batch(grid, tx.TX30, batch=5)
    net = pf.TxNetwork.from_grid(ctx, grid)
    ref = _solve(net, batch)
    # empty batch
    e = torch.zeros((0, grid.n_bus), dtype=torch.float64, device="cuda")
    out = net.solve(e, e, e)
    assert out.v.shape == (0, grid.n_bus)
    # padded rows (ld > n)
    ld = grid.n_bus + 7
    pad = lambda a: to_dev(np.pad(a, ((0, 0), (0, 7))))[:, :grid.n_bus]  # noqa: E731
    res_pad = net.solve(pad(batch.p_inj), pad(batch.q_inj), pad(batch.vm_set),
                        out=pf.TxResult(v=torch.zeros((5, ld), dtype=torch.complex128, device="cuda")[:, :grid.n_bus],
                                        newton_iters=torch.empty(5, dtype=torch.int32, device="cuda"),
                                        gmres_iters=torch.empty(5, dtype=torch.int32, device="cuda"),
                                        converged=torch.empty(5, dtype=torch.uint8, device="cuda"),
                                        mismatch=torch.empty(5, dtype=torch.float64, device="cuda")))
    torch.cuda.synchronize()
    assert torch.equal(res_pad.v, ref.v)
    # bad scenarios next to good ones
    p = batch.p_inj.copy()
    q = batch.q_inj.copy()
    p[1] *= 50
    q[1] *= 50
    p[3, 4] = np.nan
    bad = net.solve(to_dev(p), to_dev(q), to_dev(batch.vm_set))
    torch.cuda.synchronize()
    conv = bad.converged.cpu().numpy()
    assert conv[1] == 0 and conv[3] == 0 and conv[[0, 2, 4]].all()
    for c in (0, 2, 4):
        assert torch.equal(bad.v[c], ref.v[c])
    capped = _solve(net, batch, max_newton=1)
    assert not capped.converged.cpu().numpy().any()
    assert (capped.newton_iters.cpu().numpy() == 1).all()
    net.close()


def test_batch_invariance(ctx):
    """A scenario solved alone equals the same scenario inside a batch, bit for bit."""
    import torch
    from paper_2605_14103_amd import pf
    grid = tx.make_grid(tx.TX2000)
    batch = tx.make_batch(grid, tx.TX2000, batch=16)
    net = pf.TxNetwork.from_grid(ctx, grid)
    full = _solve(net, batch)
    for c in (0, 9):
        one = tx.TxBatch(batch.p_inj[c:c + 1], batch.q_inj[c:c + 1], batch.vm_set[c:c + 1])
        alone = _solve(net, one)
        assert torch.equal(alone.v[0], full.v[c])
    again = _solve(net, batch)
    assert torch.equal(again.v, full.v)
    net.close()


def test_block_jacobi_option_reaches_same_solution(ctx):
    from paper_2605_14103_amd import pf
    grid = tx.make_grid(tx.TX2000)
    batch = tx.make_batch(grid, tx.TX2000, batch=4)
    net = pf.TxNetwork.from_grid(ctx, grid, precond_block=64)
    res = _solve(net, batch)
    say("block-Jacobi(64) gmres its", res.gmres_iters.cpu().numpy().tolist())
    _check_against_oracle(grid, batch, res, np.arange(4), "fp64-bj64")
    net.close()


def test_branch_loss_and_gradient(ctx):
    from paper_2605_14103_amd import pf
    grid = tx.make_grid(tx.TX30)
    rng = np.random.default_rng(7)
    V = rng.uniform(0.9, 1.1, (3, grid.n_bus)) * np.exp(1j * rng.uniform(-0.2, 0.2, (3, grid.n_bus)))
    net = pf.TxNetwork.from_grid(ctx, grid)
    loss, g = net.branch_loss(to_dev(V))
    Lref = oadj.branch_loss(grid, V.T)
    gref = np.conj(oadj.branch_loss_grad(grid, V.T)).T   # torch convention
    np.testing.assert_allclose(loss.cpu().numpy(), Lref, rtol=1e-12)
    np.testing.assert_allclose(g.cpu().numpy(), gref, rtol=1e-11, atol=1e-11)
    net.close()


@pytest.mark.parametrize("cfg,cols", [(tx.TX30, [0, 5]), (tx.TX2000_ADJ, [0, 255])])
def test_adjoint_matches_dense_adjoint(ctx, cfg, cols):
    from paper_2605_14103_amd import pf
    say("adjoint", cfg.name)
    grid = tx.make_grid(cfg)
    batch = tx.make_batch(grid, cfg)
    net = pf.TxNetwork.from_grid(ctx, grid)
    res = _solve(net, batch, tol=1e-11)
    loss, g = net.branch_loss(res.v)
    gp, gq, its, ok = net.adjoint(res.v, g)
    gp = gp.cpu().numpy()
    gq = gq.cpu().numpy()
    assert ok.cpu().numpy().all()
    V = res.v.cpu().numpy()
    for c in cols:
        rp, rq = oadj.dense_adjoint(grid, V[c])
        scale = max(np.abs(rp).max(), np.abs(rq).max())
        err = max(np.abs(gp[c] - rp).max(), np.abs(gq[c] - rq).max()) / scale
        say(f"adjoint {cfg.name} scenario {c}: rel err {err:.2e}, gmres {int(its[c])}")
        assert err <= 1e-8
    net.close()


def test_autograd_matches_finite_differences(ctx):
    """Gradient of a torch loss on the solved voltages through the adjoint, against
    central differences of the oracle's solves (h = 1e-6, solves to 1e-12)."""
    import torch
    from oracle import nr as onr
    from paper_2605_14103_amd import autograd, pf
    grid = tx.make_grid(tx.TX30)
    batch = tx.make_batch(grid, tx.TX30, batch=2)
    net = pf.TxNetwork.from_grid(ctx, grid)
    p = to_dev(batch.p_inj).requires_grad_(True)
    q = to_dev(batch.q_inj).requires_grad_(True)
    vm = to_dev(batch.vm_set)
    v, conv = autograd.solve(net, p, q, vm, tol=1e-12)
    f = torch.from_numpy(grid.f.astype(np.int64)).cuda()
    t = torch.from_numpy(grid.t.astype(np.int64)).cuda()
    ys = torch.from_numpy(1.0 / (grid.r + 1j * grid.x)).cuda()
    yff = ys + 0.5j * torch.from_numpy(grid.b).cuda()
    i_f = yff * v[:, f] - ys * v[:, t]
    loss = (i_f.abs() ** 2).sum()
    loss.backward()
    gp = p.grad.cpu().numpy()
    gq = q.grad.cpu().numpy()
    Y = onr.ybus(grid.n_bus, grid.f, grid.t, grid.r, grid.x, grid.b)

    def L(pp, qq, c):
        r = onr.nr_solve(Y, grid.bus_type, pp, qq, batch.vm_set[c], tol=1e-13)
        vv = r.V
        return float(np.sum(np.abs((1 / (grid.r + 1j * grid.x) + 0.5j * grid.b) * vv[grid.f]
                                   - (1 / (grid.r + 1j * grid.x)) * vv[grid.t]) ** 2))

    h = 1e-6
    theta = np.flatnonzero(grid.bus_type != tx.SLACK)
    pq = np.flatnonzero(grid.bus_type == tx.PQ)
    scale = max(np.abs(gp).max(), np.abs(gq).max())
    for c in range(2):
        for k in theta[::5]:
            e = np.zeros(grid.n_bus)
            e[k] = h
            fd = (L(batch.p_inj[c] + e, batch.q_inj[c], c) - L(batch.p_inj[c] - e, batch.q_inj[c], c)) / (2 * h)
            assert abs(fd - gp[c, k]) <= 1e-5 * scale
        for k in pq[::5]:
            e = np.zeros(grid.n_bus)
            e[k] = h
            fd = (L(batch.p_inj[c], batch.q_inj[c] + e, c) - L(batch.p_inj[c], batch.q_inj[c] - e, c)) / (2 * h)
            assert abs(fd - gq[c, k]) <= 1e-5 * scale
        assert gp[c, grid.slack] == 0 and np.all(gq[c, grid.bus_type != tx.PQ] == 0)
    net.close()


# One grid per workgroup shape of the solve kernels: (64 threads, 1 slot),
# (64, 4), (256, 4), (512, 8) and (1024, 8); the 2000-bus grid above covers
# (256, 8).  Three scenarios each (the 8000-bus grid checks one against the
# oracle, whose sparse solve takes seconds there).
@pytest.mark.parametrize("n_bus,n_check", [(50, 3), (200, 3), (700, 3), (3000, 3), (8000, 1)])
def test_every_workgroup_shape(ctx, n_bus, n_check):
    from paper_2605_14103_amd import pf
    cfg = tx.TxConfig(f"tx{n_bus}", n_bus=n_bus, n_pv=max(1, (3 * n_bus) // 20), n_branch=(13 * n_bus) // 10,
                      batch=3, seed=n_bus, perturbation="uniform", spread=0.2)
    say(cfg.name)
    grid = tx.make_grid(cfg)
    batch = tx.make_batch(grid, cfg)
    net = pf.TxNetwork.from_grid(ctx, grid)
    for precision in ("fp64", "mixed"):
        res = _solve(net, batch, precision=pf.precision(precision))
        assert res.converged.cpu().numpy().all()
        _check_against_oracle(grid, batch, res, np.arange(n_check), precision)
    net.close()


def _solve_yvals(net, batch, yv, **opts):
    import torch
    res = net.solve_yvals(to_dev(batch.p_inj), to_dev(batch.q_inj), to_dev(batch.vm_set), yv, **opts)
    torch.cuda.synchronize()
    return res


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_yvals_with_the_networks_own_values_is_bitwise_the_shared_solve(ctx, precision):
    """Per-scenario values equal to the network's own (tiled, in rows padded past
    nnz) give the shared-value solve bit for bit: same layout, same arithmetic."""
    import torch
    from paper_2605_14103_amd import pf
    for cfg, B in ((tx.TX30, 64), (tx.TX2000, 48)):
        grid = tx.make_grid(cfg)
        batch = tx.make_batch(grid, cfg, batch=B)
        net = pf.TxNetwork.from_grid(ctx, grid)
        base = net.csr[2] + 1j * net.csr[3]
        nnz = base.shape[0]
        yv = torch.zeros((B, nnz + 5), dtype=torch.complex128)
        yv[:, :nnz] = torch.from_numpy(base)[None, :]
        yv = yv.cuda()[:, :nnz]
        say(f"{cfg.name} yvals identity {precision}: nnz {nnz}, ldy {yv.stride(0)}")
        ref = _solve(net, batch, precision=pf.precision(precision))
        res = _solve_yvals(net, batch, yv, precision=pf.precision(precision))
        assert torch.equal(res.v, ref.v)
        assert torch.equal(res.newton_iters, ref.newton_iters)
        assert torch.equal(res.gmres_iters, ref.gmres_iters)
        assert torch.equal(res.converged, ref.converged)
        assert torch.equal(res.mismatch, ref.mismatch)
        # the byte model adds the scenario's Ybus entries
        assert (res.work_bytes > ref.work_bytes).all()
        net.close()


def _check_outages(grid, batch, on, res, cols, label):
    v = res.v.cpu().numpy()
    conv = res.converged.cpu().numpy()
    mis = res.mismatch.cpu().numpy()
    errs = []
    for c in cols:
        m = on[c].astype(bool)
        Y = onr.ybus(grid.n_bus, grid.f[m], grid.t[m], grid.r[m], grid.x[m], grid.b[m])
        ref = onr.nr_solve(Y, grid.bus_type, batch.p_inj[c], batch.q_inj[c], batch.vm_set[c])
        assert ref.converged, f"oracle did not converge for scenario {c}"
        assert conv[c] and mis[c] <= 1e-8
        errs.append(angle_err(v[c:c + 1], ref.V[None, :]))
    da = max(e[0] for e in errs)
    dm = max(e[1] for e in errs)
    say(f"{label}: {len(cols)} scenarios, max angle err {da:.2e} rad, max |V| err {dm:.2e} pu, "
        f"newton {res.newton_iters.cpu().numpy()[cols].tolist()[:8]}, "
        f"gmres {res.gmres_iters.cpu().numpy()[cols].tolist()[:8]}")
    assert da <= TOL_A and dm <= TOL_V


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_branch_outages_against_oracle(ctx, precision):
    """Topology-action batches: every scenario of the 30-bus grid with two
    branches out, and sampled scenarios of the 2000-bus grid with one branch out
    at batch 1024, each against the oracle solving with that scenario's own
    admittance matrix."""
    import torch
    from paper_2605_14103_amd import pf
    for cfg, n_out, cols in ((tx.TX30, 2, None), (tx.TX2000, 1, spread_cols(tx.TX2000.batch, 32))):
        grid = tx.make_grid(cfg)
        batch = tx.make_batch(grid, cfg)
        on = tx.make_outages(grid, batch.batch, n_out=n_out, seed=cfg.seed + 7)
        net = pf.TxNetwork.from_grid(ctx, grid)
        yv = torch.from_numpy(net.ybus_switch(on)).cuda()
        res = _solve_yvals(net, batch, yv, precision=pf.precision(precision))
        conv = res.converged.cpu().numpy().astype(bool)
        say(f"{cfg.name} outages {precision}: converged {int(conv.sum())} of {batch.batch}")
        # Every converged scenario reached the high-voltage solution: those
        # above the floor by the floor, and the few that an outage leaves
        # below it (a bus fed over a long path after its line is switched
        # out) by the oracle's own flat-start solve, element by element.  The
        # outages that leave no solution near flat start report converged = 0.
        vmin = np.abs(res.v.cpu().numpy()).min(axis=1)
        low = np.where(conv & ~(vmin > HV_FLOOR_TX))[0]
        say(f"{cfg.name} outages {precision}: {len(low)} converged scenarios below {HV_FLOOR_TX} pu: "
            f"{low.tolist()} at {np.round(vmin[low], 4).tolist()}")
        assert len(low) <= 8, "more sagging scenarios than the oracle check is sized for"
        assert_high_voltage(res.v.cpu().numpy()[conv & (vmin > HV_FLOOR_TX)], HV_FLOOR_TX, f"{cfg.name} outages")
        check = np.arange(batch.batch) if cols is None else np.union1d(cols, low)
        _check_outages(grid, batch, on, res, check, f"{cfg.name} {n_out} out {precision}")
        net.close()


def test_yvals_argument_errors(ctx):
    import torch
    from paper_2605_14103_amd import _lib, pf
    grid = tx.make_grid(tx.TX30)
    batch = tx.make_batch(grid, tx.TX30, batch=4)
    net = pf.TxNetwork.from_grid(ctx, grid)
    nnz = net.csr[1].shape[0]
    with pytest.raises(ValueError):  # rows shorter than nnz
        _solve_yvals(net, batch, torch.zeros((4, nnz - 1), dtype=torch.complex128, device="cuda"))
    with pytest.raises(ValueError):  # one row per scenario
        _solve_yvals(net, batch, torch.zeros((3, nnz), dtype=torch.complex128, device="cuda"))
    # the C entry point itself rejects ldy < nnz and a null y_vals
    o = _lib.opts()
    import ctypes
    st = _lib.lib().pf_tx_solve_yvals(net.h, ctypes.byref(o), 0, grid.n_bus, None, None, None, nnz - 1, None,
                                      None, None, None, None, None, None, None)
    assert st == _lib.PF_INVALID_ARG
    p = to_dev(batch.p_inj)
    st = _lib.lib().pf_tx_solve_yvals(net.h, ctypes.byref(o), 4, grid.n_bus, ctypes.c_void_p(p.data_ptr()),
                                      ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(p.data_ptr()), nnz, None,
                                      None, None, None, None, None, None, None)
    assert st == _lib.PF_INVALID_ARG
    net.close()


def _grid_cfg(n_bus):
    if n_bus == 30:
        return tx.TX30
    return tx.TxConfig(f"tx{n_bus}", n_bus=n_bus, n_pv=max(5, n_bus * 15 // 100), n_branch=int(n_bus * 1.3),
                       batch=48, seed=n_bus, perturbation="uniform", spread=0.2)


@pytest.mark.parametrize("n_bus", [30, 118, 500])
def test_direct_newton_matches_oracle_step_for_step(ctx, n_bus):
    """The direct Newton step (per-scenario sparse LU on the shared analysis)
    takes exact Newton steps, as the oracle does: every scenario agrees with the
    oracle in V and takes the same number of Newton updates."""
    from paper_2605_14103_amd import pf
    cfg = _grid_cfg(n_bus)
    grid = tx.make_grid(cfg)
    batch = tx.make_batch(grid, cfg)
    net = pf.TxNetwork.from_grid(ctx, grid)
    res = _solve(net, batch, nr_direct=1)
    V, it, ok, mm = onr.nr_solve_batch(grid, batch)
    v = res.v.cpu().numpy()
    da, dm = angle_err(v, V)
    nit = res.newton_iters.cpu().numpy()
    say(f"{cfg.name} direct: max angle err {da:.2e}, max |V| err {dm:.2e}, newton {nit.tolist()[:8]} "
        f"(oracle {it.tolist()[:8]}), mismatch max {res.mismatch.cpu().numpy().max():.2e}")
    assert ok.all() and res.converged.cpu().numpy().all()
    assert res.mismatch.cpu().numpy().max() <= 1e-8
    assert da <= TOL_A and dm <= TOL_V
    np.testing.assert_array_equal(nit, it)
    assert (res.gmres_iters.cpu().numpy() == 0).all()
    net.close()


def test_direct_newton_with_branch_outages(ctx):
    """The direct step with per-scenario admittance values: the 30-bus grid with
    two branches out per scenario against the oracle (same Newton updates)."""
    import torch
    from paper_2605_14103_amd import pf
    grid = tx.make_grid(tx.TX30)
    batch = tx.make_batch(grid, tx.TX30)
    on = tx.make_outages(grid, batch.batch, n_out=2, seed=37)
    net = pf.TxNetwork.from_grid(ctx, grid)
    yv = torch.from_numpy(net.ybus_switch(on)).cuda()
    res = _solve_yvals(net, batch, yv, nr_direct=1)
    _check_outages(grid, batch, on, res, np.arange(batch.batch), "tx30 direct, 2 out")
    nit = res.newton_iters.cpu().numpy()
    for c in range(batch.batch):
        m = on[c].astype(bool)
        Y = onr.ybus(grid.n_bus, grid.f[m], grid.t[m], grid.r[m], grid.x[m], grid.b[m])
        ref = onr.nr_solve(Y, grid.bus_type, batch.p_inj[c], batch.q_inj[c], batch.vm_set[c])
        assert nit[c] == ref.iters
    net.close()


def test_direct_newton_on_the_2000_bus_grid(ctx):
    """The 2000-bus grid's factor (36 k values per scenario) does not fit LDS
    and lives in device memory: at its full batch of 1024 every scenario
    converges, and spread scenarios agree with the oracle in V and in the
    number of Newton updates (both take exact Newton steps)."""
    from paper_2605_14103_amd import pf
    grid = tx.make_grid(tx.TX2000)
    batch = tx.make_batch(grid, tx.TX2000)
    net = pf.TxNetwork.from_grid(ctx, grid)
    res = _solve(net, batch, nr_direct=1)
    conv = res.converged.cpu().numpy()
    nit = res.newton_iters.cpu().numpy()
    say(f"tx2000 direct: converged {int(conv.sum())} of {batch.batch}, newton {np.bincount(nit).tolist()}, "
        f"mismatch max {res.mismatch.cpu().numpy().max():.2e}")
    assert conv.all() and res.mismatch.cpu().numpy().max() <= 1e-8
    assert_high_voltage(res.v.cpu().numpy(), HV_FLOOR_TX, "tx2000 direct")
    cols = spread_cols(batch.batch, 32)
    V, it, ok, _ = onr.nr_solve_batch(grid, batch, columns=cols)
    da, dm = angle_err(res.v.cpu().numpy()[cols], V)
    say(f"tx2000 direct: max angle err {da:.2e}, max |V| err {dm:.2e}")
    assert ok.all() and da <= TOL_A and dm <= TOL_V
    np.testing.assert_array_equal(nit[cols], it)
    # the GMRES path on the same network afterwards gives the same solutions
    g = _solve(net, batch)
    da, dm = angle_err(g.v.cpu().numpy(), res.v.cpu().numpy())
    assert g.converged.cpu().numpy().all() and da <= 2 * TOL_A and dm <= 2 * TOL_V
    net.close()


def test_direct_newton_refuses_a_network_too_large(ctx):
    """Above 2048 buses the LDS no longer holds V, I, the right-hand side and
    x of one scenario: the direct step is refused, the network stays usable."""
    from paper_2605_14103_amd import _lib, pf
    cfg = tx.TxConfig("tx3000", n_bus=3000, n_pv=450, n_branch=3900, batch=2, seed=3000,
                      perturbation="uniform", spread=0.2)
    grid = tx.make_grid(cfg)
    batch = tx.make_batch(grid, cfg, batch=2)
    net = pf.TxNetwork.from_grid(ctx, grid)
    with pytest.raises(_lib.PfError) as e:
        _solve(net, batch, nr_direct=1)
    assert e.value.status == _lib.PF_INVALID_ARG and "too large for the direct Newton step" in str(e.value)
    # the GMRES path still works on the same network afterwards
    res = _solve(net, batch)
    assert res.converged.cpu().numpy().all()
    net.close()


def test_direct_edge_cases_and_isolation(ctx):
    """The direct step: empty batch, an infeasible and a NaN scenario next to
    good ones (the good ones bitwise unaffected), an iteration cap of one."""
    import torch
    from paper_2605_14103_amd import pf
    grid = tx.make_grid(tx.TX30)
    batch = tx.make_batch(grid, tx.TX30, batch=5)
    net = pf.TxNetwork.from_grid(ctx, grid)
    ref = _solve(net, batch, nr_direct=1)
    e = torch.zeros((0, grid.n_bus), dtype=torch.float64, device="cuda")
    assert net.solve(e, e, e, nr_direct=1).v.shape == (0, grid.n_bus)
    p = batch.p_inj.copy()
    q = batch.q_inj.copy()
    p[1] *= 50
    q[1] *= 50
    p[3, 4] = np.nan
    bad = net.solve(to_dev(p), to_dev(q), to_dev(batch.vm_set), nr_direct=1)
    torch.cuda.synchronize()
    conv = bad.converged.cpu().numpy()
    assert conv[1] == 0 and conv[3] == 0 and conv[[0, 2, 4]].all()
    for c in (0, 2, 4):
        assert torch.equal(bad.v[c], ref.v[c])
    capped = _solve(net, batch, max_newton=1, nr_direct=1)
    assert not capped.converged.cpu().numpy().any()
    assert (capped.newton_iters.cpu().numpy() == 1).all()
    # the direct step ignores the precision option (always FP64): same result
    mixed = _solve(net, batch, nr_direct=1, precision=pf.precision("mixed"))
    assert torch.equal(mixed.v, ref.v)
    net.close()


def test_adjoint_tx2000_against_central_differences(ctx):
    """The sensitivity workload at full shape: the 2000-bus grid, batch 256,
    GPU gradients of the branch loss with respect to 64 seeded injections (32 P
    on Theta buses, 32 Q on PQ buses) in 4 scenarios, against central
    differences (h = 1e-6) of the oracle's solves.  Each perturbed solve takes
    two exact Newton steps from the unperturbed solution, which drives it to
    rounding level (quadratic convergence from 1e-6 away), as the check needs."""
    from paper_2605_14103_amd import pf
    cfg = tx.TX2000_ADJ
    grid = tx.make_grid(cfg)
    batch = tx.make_batch(grid, cfg)
    net = pf.TxNetwork.from_grid(ctx, grid)
    res = _solve(net, batch, tol=1e-11)
    assert res.converged.cpu().numpy().all()
    loss, g = net.branch_loss(res.v)
    gp, gq, its, ok = net.adjoint(res.v, g)
    assert ok.cpu().numpy().all()
    gp = gp.cpu().numpy()
    gq = gq.cpu().numpy()
    Y = onr.ybus(grid.n_bus, grid.f, grid.t, grid.r, grid.x, grid.b)
    theta = np.flatnonzero(grid.bus_type != tx.SLACK)
    pq = np.flatnonzero(grid.bus_type == tx.PQ)
    rng = np.random.default_rng(2024)
    p_idx = rng.choice(theta, 32, replace=False)
    q_idx = rng.choice(pq, 32, replace=False)
    h = 1e-6
    for c in (0, 85, 170, 255):
        p0, q0, vs = batch.p_inj[c], batch.q_inj[c], batch.vm_set[c]
        base = onr.nr_solve(Y, grid.bus_type, p0, q0, vs, tol=1e-12)
        assert base.mismatch <= 1e-10

        def L(pp, qq):
            r = onr.nr_solve(Y, grid.bus_type, pp, qq, vs, tol=0.0, max_iter=2, V0=base.V)
            assert r.mismatch <= 1e-10
            return float(oadj.branch_loss(grid, r.V))

        scale = max(np.abs(gp[c]).max(), np.abs(gq[c]).max())
        worst = 0.0
        for k in p_idx:
            e = np.zeros(grid.n_bus)
            e[k] = h
            fd = (L(p0 + e, q0) - L(p0 - e, q0)) / (2 * h)
            worst = max(worst, abs(fd - gp[c, k]) / scale)
        for k in q_idx:
            e = np.zeros(grid.n_bus)
            e[k] = h
            fd = (L(p0, q0 + e) - L(p0, q0 - e)) / (2 * h)
            worst = max(worst, abs(fd - gq[c, k]) / scale)
        say(f"tx2000 adjoint vs central differences, scenario {c}: max err {worst:.2e} of max |grad| "
            f"{scale:.3e}, adjoint gmres {int(its[c])}")
        assert worst <= 1e-5
    net.close()


def test_autograd_reports_nonconvergence(ctx):
    """A backward pass through a scenario whose forward solve or adjoint solve
    did not converge raises (the default) or, with on_failure="zero", warns and
    returns zero gradient rows for it; a converged batch passes."""
    from paper_2605_14103_amd import autograd, pf
    grid = tx.make_grid(tx.TX30)
    batch = tx.make_batch(grid, tx.TX30, batch=3)
    net = pf.TxNetwork.from_grid(ctx, grid)

    def run(**kw):
        p = to_dev(batch.p_inj).requires_grad_(True)
        q = to_dev(batch.q_inj).requires_grad_(True)
        v, conv = autograd.solve(net, p, q, to_dev(batch.vm_set), **kw)
        (v.abs() ** 2).sum().backward()
        return p.grad.cpu().numpy(), q.grad.cpu().numpy()

    # adjoint starved: one Arnoldi step in one cycle cannot reach its 1e-10 tolerance
    with pytest.raises(autograd.NonConvergedGradient) as e:
        run(adjoint_opts={"gmres_restart": 1, "gmres_max_restarts": 1})
    assert e.value.adjoint_failed and not e.value.forward_failed
    # forward capped at one Newton update: no scenario converges
    with pytest.raises(autograd.NonConvergedGradient) as e:
        run(max_newton=1)
    assert e.value.forward_failed == [0, 1, 2]
    with pytest.warns(RuntimeWarning):
        gp, gq = run(max_newton=1, on_failure="zero")
    assert (gp == 0).all() and (gq == 0).all()
    gp, gq = run()
    assert np.abs(gp).max() > 0 and np.isfinite(gp).all() and np.isfinite(gq).all()
    net.close()
