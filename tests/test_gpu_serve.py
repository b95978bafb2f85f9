"""Serving engine on the GPU: admission by HBM footprint, step-level continuous
batching over several streams, caller-driven admit / step / harvest, and
results identical, bit for bit, to the same scenarios solved alone."""
import time

import numpy as np
import pytest

from oracle import nr as onr
from oracle import zbus as ozb
from tests.gpu_common import angle_err, say, to_dev
from workloads import feeder as fdm
from workloads import serving as wsv
from workloads import transmission as tx

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2605_14103_amd import pf
    assert torch.cuda.is_available()
    c = pf.Context(0)
    yield c
    c.close()


def _collect(eng, ids, timeout=60.0):
    out = {}
    deadline = time.time() + timeout
    while len(out) < len(ids) and time.time() < deadline:
        for rid in eng.poll(64, 0.01):
            out[rid] = eng.fetch(rid)
    assert len(out) == len(ids), f"only {len(out)} of {len(ids)} requests finished"
    return out


def _alone_tx(net, p, q, vm, **opts):
    import torch
    r = net.solve(to_dev(p), to_dev(q), to_dev(vm), **opts)
    torch.cuda.synchronize()
    return r.v.cpu().numpy(), r.newton_iters.cpu().numpy(), r.converged.cpu().numpy()


def _alone_dist(net, sw, sd, **opts):
    import torch
    r = net.solve(to_dev(sw), to_dev(sd), **opts)
    torch.cuda.synchronize()
    return r.v.cpu().numpy(), r.iters.cpu().numpy(), r.converged.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tx_alone_equals_mix(ctx, precision):
    """Requests submitted back to back share step launches on two streams;
    every scenario must equal, bit for bit, the same request solved alone."""
    from paper_2605_14103_amd import pf
    say("serve tx30", precision)
    grid = tx.make_grid(tx.TX30)
    net = pf.TxNetwork.from_grid(ctx, grid)
    prec = pf.precision(precision)
    sizes = [1, 7, 33, 2, 64, 5, 17, 40, 3, 9, 12, 1]
    reqs = [tx.make_batch(grid, tx.TX30, batch=n, seed=100 + i) for i, n in enumerate(sizes)]
    eng = pf.Engine(net, hbm_bytes=1 << 30, n_streams=2, precision=prec)
    say("engine", eng.info())
    for i, b in enumerate(reqs):
        eng.submit(i, b.p_inj, b.q_inj, b.vm_set)
    got = _collect(eng, list(range(len(reqs))))
    info = eng.info()
    say("after", info)
    steps_alone = 0
    for i, b in enumerate(reqs):
        v, it, ok = _alone_tx(net, b.p_inj, b.q_inj, b.vm_set, precision=prec)
        steps_alone += int(it.max()) + 1
        r = got[i]
        assert r.converged.all() and ok.all()
        assert np.array_equal(r.v.view(np.float64), v.view(np.float64)), f"request {i} differs from alone"
        assert np.array_equal(r.iters, it)
        assert r.mismatch.max() <= 1e-8
        assert r.times[0] <= r.times[1] <= r.times[2]
    assert info["steps"] < steps_alone, "requests did not share steps"
    assert info["occupied"] == 0 and info["scenarios"] == sum(sizes)
    # and the mix against the oracle for a few requests
    for i in (1, 4):
        V, _, ok, _ = onr.nr_solve_batch(grid, reqs[i])
        da, dm = angle_err(got[i].v, V)
        assert ok.all() and da <= 1e-6 and dm <= 1e-6
    eng.close()
    net.close()


@pytest.mark.parametrize("sparse", [0, 1])
def test_feeder_alone_equals_mix(ctx, sparse):
    from paper_2605_14103_amd import pf
    say("serve feeder40, sparse update" if sparse else "serve feeder40")
    cfg = fdm.FeederConfig("feeder40", n_bus=40, max_depth=25, batch=1, seed=41)
    fd = fdm.make_feeder(cfg)
    net = pf.DistNetwork.from_feeder(ctx, fd)
    sizes = [3, 130, 1, 64, 200, 7, 129, 2]
    reqs = [fdm.make_batch(fd, cfg, batch=n, seed=500 + i) for i, n in enumerate(sizes)]
    eng = pf.Engine(net, hbm_bytes=64 << 20, n_streams=2, zbus_sparse=sparse)
    say("engine", eng.info())
    for i, b in enumerate(reqs):
        eng.submit(i, b.s_wye, b.s_delta)
    got = _collect(eng, list(range(len(reqs))))
    say("after", eng.info())
    for i, b in enumerate(reqs):
        v, it, ok = _alone_dist(net, b.s_wye, b.s_delta, zbus_sparse=sparse)
        r = got[i]
        assert r.converged.all() and ok.all()
        assert np.array_equal(r.v.view(np.float64), v.view(np.float64)), f"request {i} differs from alone"
        assert np.array_equal(r.iters, it)
    ref = ozb.zbus_solve(fd, reqs[0])
    da, dm = angle_err(got[0].v, ref.v)
    assert da <= 1e-6 and dm <= 1e-6
    eng.close()
    net.close()


def test_admission_limits_and_lifetime(ctx):
    from paper_2605_14103_amd import _lib as L
    from paper_2605_14103_amd import pf
    grid = tx.make_grid(tx.TX30)
    net = pf.TxNetwork.from_grid(ctx, grid)
    probe = pf.Engine(net, hbm_bytes=1 << 24, n_streams=1)
    slot = probe.slot_bytes
    probe.close()
    with pytest.raises(L.PfError) as e:
        pf.Engine(net, hbm_bytes=slot - 1)
    assert e.value.status == L.PF_INVALID_ARG
    with pytest.raises(L.PfError) as e:  # the engine runs the GMRES step only
        pf.Engine(net, hbm_bytes=4 * slot, nr_direct=1)
    assert e.value.status == L.PF_INVALID_ARG and "nr_direct" in str(e.value)
    eng = pf.Engine(net, hbm_bytes=4 * slot, n_streams=1)
    assert eng.info()["max_slots"] == 4
    b = tx.make_batch(grid, tx.TX30, batch=5, seed=1)
    with pytest.raises(L.PfError) as e:
        eng.submit(0, b.p_inj, b.q_inj, b.vm_set)
    assert e.value.status == L.PF_NOT_ADMITTED
    # three requests of 3 slots on a 4-slot engine: each waits for slots the
    # one before it frees, and they are admitted in arrival order
    for i in range(3):
        eng.submit(10 + i, b.p_inj[:3], b.q_inj[:3], b.vm_set[:3])
    got = _collect(eng, [10, 11, 12])
    assert all(r.converged.all() for r in got.values())
    adm = [got[10 + i].times[1] for i in range(3)]
    assert adm[0] <= adm[1] <= adm[2]
    assert got[10].times[1] < got[11].times[1], "the second request was admitted with the first"
    # the request-driven engine refuses the caller-driven calls
    with pytest.raises(L.PfError) as e:
        eng.admit([0], b.p_inj[:1], b.q_inj[:1], b.vm_set[:1])
    assert e.value.status == L.PF_INVALID_ARG
    eng.submit(20, b.p_inj[:1], b.q_inj[:1], b.vm_set[:1])
    with pytest.raises(L.PfError) as e:
        eng.submit(20, b.p_inj[:1], b.q_inj[:1], b.vm_set[:1])
    assert e.value.status == L.PF_INVALID_ARG
    _collect(eng, [20])
    # destroying the network takes the engine with it
    net.close()
    with pytest.raises(L.PfError) as e:
        eng.info()
    assert e.value.status == L.PF_BAD_HANDLE
    eng.h = None


def test_short_trace_replay(ctx):
    """A compressed Poisson trace over two grids and a feeder; everything converges."""
    from paper_2605_14103_amd import pf, serve
    say("serve replay")
    g30 = tx.make_grid(tx.TX30)
    cfg_f = fdm.FeederConfig("feeder40", n_bus=40, max_depth=25, batch=1, seed=41)
    fd = fdm.make_feeder(cfg_f)
    cfg_b = tx.TxConfig("tx200", n_bus=200, n_pv=30, n_branch=260, batch=1, seed=200,
                        perturbation="uniform", spread=0.2)
    g200 = tx.make_grid(cfg_b)
    nets = [pf.TxNetwork.from_grid(ctx, g30), pf.TxNetwork.from_grid(ctx, g200), pf.DistNetwork.from_feeder(ctx, fd)]
    engines = [pf.Engine(n, hbm_bytes=256 << 20, n_streams=s) for n, s in zip(nets, (1, 2, 1))]
    trace = wsv.make_trace(wsv.ServingConfig(lam=4000.0, n_requests=60, max_scen=64, n_networks=3, seed=11))

    def inputs(r):
        if r.network == 0:
            b = tx.make_batch(g30, tx.TX30, batch=r.n_scen, seed=r.seed)
            return b.p_inj, b.q_inj, b.vm_set
        if r.network == 1:
            b = tx.make_batch(g200, cfg_b, batch=r.n_scen, seed=r.seed)
            return b.p_inj, b.q_inj, b.vm_set
        b = fdm.make_batch(fd, cfg_f, batch=r.n_scen, seed=r.seed)
        return b.s_wye, b.s_delta

    st = serve.replay(engines, trace, inputs, timeout_s=60)
    summ = st.summary()
    say("replay", {k: v for k, v in summ.items() if k != "per_network"})
    assert not st.failed
    assert summ["converged"] == summ["scenarios"] == sum(r.n_scen for r in trace)
    for e in engines:
        e.close()
    for n in nets:
        n.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_networks_in_one_mix(ctx, precision):
    """The serving mix's own networks at full size: the 2000-bus grid and the
    900-node feeder, with the 30-bus grid, each behind its engine; requests of
    1 to 512 scenarios are submitted interleaved so that the three engines run
    at once.  Every request equals its solve alone bit for bit, and scenarios
    spread over the requests match the oracle."""
    from paper_2605_14103_amd import pf
    prec = pf.precision(precision)
    g30 = tx.make_grid(tx.TX30)
    g2k = tx.make_grid(tx.TX2000)
    fd = fdm.make_feeder(fdm.FEEDER300)
    nets = [pf.TxNetwork.from_grid(ctx, g30), pf.TxNetwork.from_grid(ctx, g2k), pf.DistNetwork.from_feeder(ctx, fd)]
    engines = [pf.Engine(n, hbm_bytes=b, n_streams=s, precision=prec)
               for n, b, s in zip(nets, (256 << 20, 4 << 30, 1 << 30), (1, 2, 1))]
    sizes = {0: [5, 64, 1], 1: [1, 37, 512, 3, 200], 2: [3, 300, 1, 129, 512]}
    reqs = []
    for k in range(max(len(v) for v in sizes.values())):
        for net_id, sz in sizes.items():
            if k < len(sz):
                seed = 900 + 10 * net_id + k
                if net_id == 0:
                    b = tx.make_batch(g30, tx.TX30, batch=sz[k], seed=seed)
                    arrays = (b.p_inj, b.q_inj, b.vm_set)
                elif net_id == 1:
                    b = tx.make_batch(g2k, tx.TX2000, batch=sz[k], seed=seed)
                    arrays = (b.p_inj, b.q_inj, b.vm_set)
                else:
                    b = fdm.make_batch(fd, fdm.FEEDER300, batch=sz[k], seed=seed)
                    arrays = (b.s_wye, b.s_delta)
                rid = len(reqs)
                reqs.append((net_id, rid, b, arrays))
                engines[net_id].submit(rid, *arrays)
    got = {}
    for net_id in range(3):
        ids = [rid for n, rid, _, _ in reqs if n == net_id]
        got.update(_collect(engines[net_id], ids, timeout=90.0))
    say(f"full-size mix {precision}:", [e.info() for e in engines])
    for net_id, rid, b, arrays in reqs:
        r = got[rid]
        if net_id == 2:
            v, it, ok = _alone_dist(nets[2], *arrays, precision=prec)
        else:
            v, it, ok = _alone_tx(nets[net_id], *arrays, precision=prec)
        assert r.converged.all() and ok.all(), f"request {rid} (network {net_id}) did not converge"
        assert r.mismatch.max() <= 1e-8
        assert np.array_equal(r.v.view(np.float64), v.view(np.float64)), f"request {rid} differs from alone"
        assert np.array_equal(r.iters, it)
    # oracle: two scenarios of every 2000-bus and feeder request (first and last)
    for net_id, rid, b, arrays in reqs:
        cols = np.unique([0, b.batch - 1] if net_id else [0])
        if net_id == 1:
            V, _, ok, _ = onr.nr_solve_batch(g2k, b, columns=cols)
        elif net_id == 2:
            ref = ozb.zbus_solve(fd, fdm.FeederBatch(b.s_wye[cols], b.s_delta[cols]))
            V, ok = ref.v, ref.converged
        else:
            V, _, ok, _ = onr.nr_solve_batch(g30, b, columns=cols)
        da, dm = angle_err(got[rid].v[cols], V)
        assert ok.all() and da <= 1e-6 and dm <= 1e-6, f"request {rid}: {da:.2e} rad, {dm:.2e} pu"
    for e in engines:
        e.close()
    for n in nets:
        n.close()


@pytest.mark.parametrize("kind", ["tx2000", "feeder300", "feeder300_sparse"])
def test_caller_driven_steps(ctx, kind):
    """Caller-driven engine: scenarios admitted between steps into scattered
    free slots, one iteration per step, harvested as they finish and their
    slots reused; every scenario equals its one-shot solve bit for bit."""
    import torch
    from paper_2605_14103_amd import _lib as L
    from paper_2605_14103_amd import pf
    say("caller-driven", kind)
    if kind == "tx2000":
        grid = tx.make_grid(tx.TX2000)
        net = pf.TxNetwork.from_grid(ctx, grid)
        batch = tx.make_batch(grid, tx.TX2000, batch=24, seed=77)
        inputs = [batch.p_inj, batch.q_inj, batch.vm_set]
        v_ref, it_ref, ok_ref = _alone_tx(net, *inputs)
    else:
        fd = fdm.make_feeder(fdm.FEEDER300)
        net = pf.DistNetwork.from_feeder(ctx, fd)
        batch = fdm.make_batch(fd, fdm.FEEDER300, batch=24, seed=77)
        inputs = [batch.s_wye, batch.s_delta]
        v_ref, it_ref, ok_ref = _alone_dist(net, *inputs, zbus_sparse=int(kind.endswith("sparse")))
    assert ok_ref.all()
    eng = pf.Engine(net, hbm_bytes=1 << 30, n_streams=0, zbus_sparse=int(kind.endswith("sparse")))
    slots_total = eng.info()["max_slots"]
    assert slots_total >= 16
    with pytest.raises(L.PfError) as e:      # caller-driven engines take no requests
        eng.submit(0, *[a[:1] for a in inputs])
    assert e.value.status == L.PF_INVALID_ARG
    stream = torch.cuda.current_stream()
    # waves of admission: scenario k goes into slot order[k]; later waves
    # reuse slots freed by earlier ones
    order = list(range(15, -1, -2)) + list(range(0, 16, 2))
    waves = [range(0, 5), range(5, 9), range(9, 16), range(16, 24)]
    free = list(order)
    where = {}
    got = {}
    steps = 0
    pending_waves = list(waves)
    with pytest.raises(L.PfError) as e:      # nothing finished yet
        eng.harvest([0], stream=stream)
    assert e.value.status == L.PF_INVALID_ARG
    while pending_waves or where:
        if pending_waves and len(free) >= len(pending_waves[0]):
            ks = list(pending_waves.pop(0))
            sl = [free.pop(0) for _ in ks]
            eng.admit(sl, *[a[ks] for a in inputs], stream=stream)
            for k, s_ in zip(ks, sl):
                where[s_] = k
            if steps == 0:
                with pytest.raises(L.PfError) as e:    # an occupied slot
                    eng.admit([sl[0]], *[a[:1] for a in inputs], stream=stream)
                assert e.value.status == L.PF_INVALID_ARG
        done, active = eng.step(1, stream=stream)
        steps += 1
        assert steps < 400
        if done:
            r = eng.harvest(done, stream=stream)
            for j, s_ in enumerate(done):
                k = where.pop(s_)
                got[k] = (r.v[j], r.iters[j], r.converged[j], r.mismatch[j])
                free.append(s_)
    say(f"{kind}: {steps} steps for 24 scenarios in 4 waves, info {eng.info()}")
    for k in range(24):
        v, it, ok, mm = got[k]
        assert ok and mm <= 1e-8
        assert np.array_equal(v.view(np.float64), v_ref[k].view(np.float64)), f"scenario {k} differs"
        assert it == it_ref[k]
    assert eng.info()["occupied"] == 0
    eng.close()
    net.close()
