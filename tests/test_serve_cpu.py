"""Trace replay and latency accounting against a CPU fake engine (no GPU).

The fake engine follows the engine interface (submit / poll / fetch / info)
and answers each request with the oracle on a tiny grid after a fixed service
delay, serving requests one at a time in FIFO order.  This checks the replay
loop's bookkeeping: every request is harvested once, latency splits into
submit lag + queue + service, throughput counts converged scenarios, a request
the engine rejects or fails is reported without disturbing the others.
"""
import threading
import time
from dataclasses import dataclass

import numpy as np
import pytest

from oracle import nr as onr
from paper_2605_14103_amd import serve
from workloads import serving as wsv
from workloads import transmission as tx


@dataclass
class FakeResult:
    v: np.ndarray
    iters: np.ndarray
    converged: np.ndarray
    mismatch: np.ndarray
    times: np.ndarray


class FakeEngine:
    def __init__(self, grid, max_slots=64, service=0.003, fail_ids=()):
        self.grid = grid
        self.max_slots = max_slots
        self.service = service
        self.fail_ids = set(fail_ids)
        self.t0 = time.perf_counter()
        self.mu = threading.Condition()
        self.queue, self.done, self.results = [], [], {}
        self.stop = False
        self.th = threading.Thread(target=self._run, daemon=True)
        self.th.start()

    def _now(self):
        return time.perf_counter() - self.t0

    def submit(self, rid, p, q, vm):
        n = p.shape[0]
        if n > self.max_slots:
            raise RuntimeError("PF_NOT_ADMITTED")
        with self.mu:
            self.queue.append((rid, tx.TxBatch(p.copy(), q.copy(), vm.copy()), self._now()))
            self.mu.notify_all()

    def _run(self):
        while True:
            with self.mu:
                while not self.queue and not self.stop:
                    self.mu.wait()
                if self.stop:
                    return
                rid, b, t_sub = self.queue.pop(0)
            t_launch = self._now()
            V, it, ok, mm = onr.nr_solve_batch(self.grid, b)
            time.sleep(self.service)
            res = FakeResult(V, it.astype(np.int32), ok.astype(np.uint8), mm,
                             np.array([t_sub, t_launch, self._now()]))
            with self.mu:
                self.results[rid] = res
                self.done.append(rid)
                self.mu.notify_all()

    def poll(self, max_ids=256, timeout=0.0):
        with self.mu:
            if not self.done and timeout > 0:
                self.mu.wait(timeout)
            out, self.done = self.done[:max_ids], self.done[max_ids:]
            return out

    def fetch(self, rid):
        with self.mu:
            res = self.results.pop(rid)
        if rid in self.fail_ids:
            raise RuntimeError("PF_HIP_ERROR: request failed")
        return res

    def info(self):
        return {"max_slots": self.max_slots}

    def close(self):
        with self.mu:
            self.stop = True
            self.mu.notify_all()
        self.th.join()


@pytest.fixture(scope="module")
def grids():
    g1, _ = tx.two_bus(0.02, 0.08, 0.5, 0.2)
    g2 = tx.make_grid(tx.TX30)
    return [g1, g2]


def _inputs(grids):
    def make(req):
        g = grids[req.network]
        if g.n_bus == 2:
            _, b = tx.two_bus(0.02, 0.08, 0.5 * (1 + 0.01 * (req.rid % 7)), 0.2, batch=req.n_scen)
            return b.p_inj, b.q_inj, b.vm_set
        b = tx.make_batch(g, tx.TX30, batch=req.n_scen, seed=req.seed)
        return b.p_inj, b.q_inj, b.vm_set
    return make


def test_replay_accounts_every_request(grids):
    cfg = wsv.ServingConfig(lam=400.0, n_requests=40, max_scen=6, n_networks=2, seed=9)
    trace = wsv.make_trace(cfg)
    engines = [FakeEngine(grids[0]), FakeEngine(grids[1])]
    try:
        st = serve.replay(engines, trace, _inputs(grids), timeout_s=30)
    finally:
        for e in engines:
            e.close()
    assert not st.failed
    assert sorted(s.rid for s in st.served) == [r.rid for r in trace]
    for s in st.served:
        assert s.queue >= 0 and s.service >= 0.003 - 1e-4
        assert s.latency >= s.queue + s.service - 1e-12
        assert s.n_converged == s.n_scen
    summ = st.summary()
    n = sum(r.n_scen for r in trace)
    assert summ["scenarios"] == n and summ["converged"] == n
    assert summ["requests"] == len(trace)
    assert 0 < summ["p50_ms"] <= summ["p99_ms"] <= summ["max_ms"]
    assert summ["max_converged_mismatch"] <= 1e-8
    # throughput over the span from the first arrival to the last completion
    assert summ["solves_per_s"] == pytest.approx(n / st.duration)
    assert set(summ["per_network"]) <= {0, 1}


def test_replay_restores_interpreter_settings_and_splits_latency(grids):
    """The replay pauses the garbage collector and shortens the thread switch
    interval only while the trace plays; the summary's latency parts are the
    submit lag, the queue and the service."""
    import gc
    import sys
    cfg = wsv.ServingConfig(lam=400.0, n_requests=10, max_scen=3, n_networks=1, seed=4)
    trace = wsv.make_trace(cfg)
    eng = FakeEngine(grids[0], service=0.001)
    switch, gc_on = sys.getswitchinterval(), gc.isenabled()
    try:
        st = serve.replay([eng], trace, _inputs(grids), timeout_s=30)
    finally:
        eng.close()
    assert sys.getswitchinterval() == switch and gc.isenabled() == gc_on
    parts = st.summary()["parts_ms"]
    assert set(parts) == {"submit_lag", "queue", "service"}
    for k, key in (("queue", "queue"), ("service", "service"), ("submit_lag", "submit_lag")):
        vals = np.array([getattr(s, key) for s in st.served]) * 1e3
        assert parts[k]["p50"] == pytest.approx(np.percentile(vals, 50))
        assert parts[k]["p99"] == pytest.approx(np.percentile(vals, 99))
    assert parts["service"]["p50"] >= 1.0 - 0.1


def test_fifo_engine_queueing_shows_in_latency(grids):
    """A burst far above the fake engine's rate queues: later requests wait longer."""
    cfg = wsv.ServingConfig(lam=1e6, n_requests=12, max_scen=1, n_networks=1, seed=3)
    trace = wsv.make_trace(cfg)
    eng = FakeEngine(grids[0], service=0.004)
    try:
        st = serve.replay([eng], trace, _inputs(grids), timeout_s=30)
    finally:
        eng.close()
    q = [s.queue for s in sorted(st.served, key=lambda s: s.rid)]
    assert q[-1] > q[0] + 0.02


def test_rejected_and_failed_requests_are_isolated(grids):
    cfg = wsv.ServingConfig(lam=500.0, n_requests=20, max_scen=8, n_networks=1, seed=5)
    trace = wsv.make_trace(cfg)
    big = [r.rid for r in trace if r.n_scen > 4]
    bad = [r.rid for r in trace if r.n_scen <= 4][:2]
    assert big and bad
    eng = FakeEngine(grids[0], max_slots=4, service=0.0, fail_ids=bad)
    try:
        st = serve.replay([eng], trace, _inputs(grids), timeout_s=30)
    finally:
        eng.close()
    failed = {rid for rid, _ in st.failed}
    assert failed == set(big) | set(bad)
    assert {s.rid for s in st.served} == {r.rid for r in trace} - failed
