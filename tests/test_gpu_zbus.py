"""Z-bus fixed point on the GPU against the CPU oracle (|v| within 1e-6 pu,
angle within 1e-6 rad, converged mismatch <= 1e-8 pu)."""
import numpy as np
import pytest

from oracle import zbus as ozb
from tests.gpu_common import HV_FLOOR_FEEDER, angle_err, assert_high_voltage, say, spread_cols, to_dev
from workloads import feeder as fdm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2605_14103_amd import pf
    assert torch.cuda.is_available()
    c = pf.Context(0)
    yield c
    c.close()


def _solve(net, batch, **opts):
    import torch
    res = net.solve(to_dev(batch.s_wye), to_dev(batch.s_delta), **opts)
    torch.cuda.synchronize()
    return res


def _check(fd, batch, res, cols, label):
    sub = fdm.FeederBatch(batch.s_wye[cols], batch.s_delta[cols])
    ref = ozb.zbus_solve(fd, sub)
    assert ref.converged.all()
    v = res.v.cpu().numpy()[cols]
    da, dm = angle_err(v, ref.v)
    mis = res.mismatch.cpu().numpy()[cols]
    its = res.iters.cpu().numpy()[cols]
    say(f"{label}: max angle err {da:.2e}, max |v| err {dm:.2e}, mismatch max {mis.max():.2e}, "
        f"iters {its.tolist()[:8]} (oracle {ref.iters.tolist()[:8]})")
    assert res.converged.cpu().numpy()[cols].all()
    assert mis.max() <= 1e-8
    assert da <= 1e-6 and dm <= 1e-6


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_small_feeder_full(ctx, precision):
    """40-bus feeder, 200 scenarios (two GEMM row tiles, ragged), all against the oracle."""
    from paper_2605_14103_amd import pf
    cfg = fdm.FeederConfig("feeder40", n_bus=40, max_depth=25, batch=200, seed=41)
    fd = fdm.make_feeder(cfg)
    batch = fdm.make_batch(fd, cfg)
    net = pf.DistNetwork.from_feeder(ctx, fd)
    res = _solve(net, batch, precision=pf.precision(precision))
    _check(fd, batch, res, np.arange(batch.batch), f"feeder40 {precision}")
    net.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_feeder300_full_batch_sampled(ctx, precision):
    from paper_2605_14103_amd import pf
    cfg = fdm.FEEDER300
    fd = fdm.make_feeder(cfg)
    batch = fdm.make_batch(fd, cfg)
    net = pf.DistNetwork.from_feeder(ctx, fd)
    say("feeder300", precision, net.info)
    res = _solve(net, batch, precision=pf.precision(precision))
    assert res.converged.cpu().numpy().all()
    assert res.mismatch.cpu().numpy().max() <= 1e-8
    assert_high_voltage(res.v.cpu().numpy(), HV_FLOOR_FEEDER, f"feeder300 {precision}")
    _check(fd, batch, res, spread_cols(batch.batch, 32), f"feeder300 {precision}")
    net.close()


@pytest.mark.parametrize("sparse", [0, 1])
@pytest.mark.parametrize("kind", [1, 2])
def test_balanced_segment_closed_form(ctx, kind, sparse):
    from paper_2605_14103_amd import pf
    from tests.test_oracle_zbus import _closed_form_phase_a
    z_self, kappa, s = 0.03 + 0.06j, 0.4, 2.0 + 0.7j
    fd, batch = fdm.single_segment(z_self, kappa, kind, s, batch=2)
    net = pf.DistNetwork.from_feeder(ctx, fd)
    res = _solve(net, batch, tol=1e-12, zbus_sparse=sparse)
    va = _closed_form_phase_a(z_self * (1 - kappa), s)
    a = np.exp(-2j * np.pi / 3)
    v = res.v.cpu().numpy()
    assert res.converged.cpu().numpy().all()
    np.testing.assert_allclose(v[:, 3:6], np.array([[va, va * a, va * a * a]] * 2), atol=1e-12)
    net.close()


@pytest.mark.parametrize("sparse", [0, 1])
def test_zero_load_and_caps(ctx, sparse):
    from paper_2605_14103_amd import pf
    cfg = fdm.FeederConfig("feeder40", n_bus=40, max_depth=25, batch=3, seed=41)
    fd = fdm.make_feeder(cfg)
    net = pf.DistNetwork.from_feeder(ctx, fd)
    res = _solve(net, fdm.zero_load(fd, 3), zbus_sparse=sparse)
    assert res.converged.cpu().numpy().all() and (res.iters.cpu().numpy() == 0).all()
    np.testing.assert_allclose(res.v.cpu().numpy(), np.tile(fd.v_slack, (3, fd.n_bus)), atol=1e-13)
    batch = fdm.make_batch(fd, cfg)
    capped = _solve(net, batch, zbus_max_iter=1, zbus_sparse=sparse)
    assert not capped.converged.cpu().numpy().any() and (capped.iters.cpu().numpy() == 1).all()
    bad = fdm.FeederBatch(batch.s_wye.copy(), batch.s_delta.copy())
    bad.s_wye[1, 5] = np.nan
    r2 = _solve(net, bad, zbus_sparse=sparse)
    full = _solve(net, batch, zbus_sparse=sparse)
    c = r2.converged.cpu().numpy()
    assert c[0] and c[2] and not c[1]
    import torch
    assert torch.equal(r2.v[0], full.v[0]) and torch.equal(r2.v[2], full.v[2])
    net.close()


def test_large_feeder_many_slots(ctx):
    """A 700-bus feeder (2097 free nodes): the residual kernel's widest slot
    template (more than 1024 free nodes per workgroup) and several GEMM column
    tiles with a ragged last one."""
    from paper_2605_14103_amd import pf
    cfg = fdm.FeederConfig("feeder700", n_bus=700, max_depth=30, batch=6, seed=700)
    fd = fdm.make_feeder(cfg)
    batch = fdm.make_batch(fd, cfg)
    net = pf.DistNetwork.from_feeder(ctx, fd)
    for precision in ("fp64", "mixed"):
        res = _solve(net, batch, precision=pf.precision(precision))
        _check(fd, batch, res, np.arange(batch.batch), f"feeder700 {precision}")
    net.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sparse_variant(ctx, precision):
    """The sparse variant (Y_NN^-1 r by the L D L^T of Y_NN instead of the dense
    Z product) against the oracle: a small feeder in full, the 300-bus feeder
    at its full batch (sampled), and 700- and 908-bus feeders (2724 phase
    nodes)."""
    from paper_2605_14103_amd import pf
    cases = [(fdm.FeederConfig("feeder40s", n_bus=40, max_depth=25, batch=33, seed=43), None),
             (fdm.FEEDER300, spread_cols(fdm.FEEDER300.batch, 32)),
             (fdm.FeederConfig("feeder700s", n_bus=700, max_depth=30, batch=5, seed=701), None),
             (fdm.FeederConfig("feeder908s", n_bus=908, max_depth=25, batch=3, seed=908), None)]
    for cfg, cols in cases:
        fd = fdm.make_feeder(cfg)
        batch = fdm.make_batch(fd, cfg)
        net = pf.DistNetwork.from_feeder(ctx, fd)
        res = _solve(net, batch, precision=pf.precision(precision), zbus_sparse=1)
        assert res.converged.cpu().numpy().all()
        assert res.mismatch.cpu().numpy().max() <= 1e-8
        assert_high_voltage(res.v.cpu().numpy(), HV_FLOOR_FEEDER, f"{cfg.name} sparse {precision}")
        _check(fd, batch, res, np.arange(batch.batch) if cols is None else cols,
               f"{cfg.name} sparse {precision}")
        dense = _solve(net, batch, precision=pf.precision(precision))
        dv = np.abs(res.v.cpu().numpy() - dense.v.cpu().numpy()).max()
        say(f"{cfg.name} sparse vs dense {precision}: max |dv| {dv:.2e}")
        assert dv <= 2e-6
        net.close()


@pytest.mark.parametrize("sparse", [0, 1])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_async_enqueue_equals_host_checked(ctx, precision, sparse):
    """All iterations enqueued at once (device-side exits) against the
    host-checked loop (the default): the same kernels on the same data, so every output
    agrees bit for bit; a second call with a smaller batch on the same
    network (its counts start from zero again) agrees too, and an iteration
    cap below convergence stops both at the same iterate."""
    import torch
    from paper_2605_14103_amd import pf
    cfg = fdm.FeederConfig("feeder120", n_bus=120, max_depth=25, batch=300, seed=121)
    fd = fdm.make_feeder(cfg)
    batch = fdm.make_batch(fd, cfg)
    net = pf.DistNetwork.from_feeder(ctx, fd)
    prec = pf.precision(precision)
    for b, extra in ((300, {}), (37, {}), (300, {"zbus_max_iter": 3})):
        sub = fdm.FeederBatch(batch.s_wye[:b], batch.s_delta[:b])
        ra = _solve(net, sub, precision=prec, zbus_sparse=sparse, zbus_async=1, **extra)
        rh = _solve(net, sub, precision=prec, zbus_sparse=sparse, zbus_async=0, **extra)
        torch.cuda.synchronize()
        for f in ("v", "iters", "converged", "mismatch", "sum_abs_change"):
            assert torch.equal(getattr(ra, f), getattr(rh, f)), f"{f} differs (batch {b}, {extra})"
        conv = ra.converged.cpu().numpy()
        say(f"async feeder120 {precision} sparse={sparse} batch {b} {extra}: converged {int(conv.sum())}, "
            f"iters max {int(ra.iters.max())}")
        assert conv.all() if not extra else not conv.any()
    _check(fd, batch, _solve(net, batch, precision=prec, zbus_sparse=sparse), spread_cols(300, 8),
           f"feeder120 async {precision} sparse={sparse}")
    net.close()
