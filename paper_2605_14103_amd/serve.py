"""Trace replay over serving engines: arrivals, harvesting and latency accounting.

The admission, slot assignment, continuous batching and stream overlap all
happen inside the native engines (``pf.Engine``); this module only plays a
request trace against them in real time: one host thread submits each
request when its arrival time comes, another harvests finished requests,
and per-request latency and throughput are recorded.

An engine here is anything with ``submit(rid, *inputs)``, ``poll(max_ids,
timeout) -> [rid]`` and ``fetch(rid)`` returning an object with ``converged``,
``mismatch`` and ``times`` (submitted, launched, completed; seconds on the
engine's own clock) fields, plus ``info()``.
"""
from __future__ import annotations

import gc
import sys
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Served:
    rid: int
    network: int
    n_scen: int
    t_arrive: float          # trace time of arrival (s)
    submit_lag: float        # host time between the arrival and the submit call (s)
    queue: float             # engine time from submit to launch (s)
    service: float           # engine time from launch to completion (s)
    n_converged: int
    max_mismatch: float
    t_done: float = 0.0      # trace time of completion (s)

    @property
    def latency(self) -> float:
        return self.submit_lag + self.queue + self.service


@dataclass
class ReplayStats:
    served: list[Served] = field(default_factory=list)
    duration: float = 0.0          # trace time from the first arrival to the last completion
    offered_span: float = 0.0      # trace time from the first to the last arrival
    failed: list[tuple[int, str]] = field(default_factory=list)

    def summary(self, tol: float = 1e-8) -> dict:
        lat = np.array([s.latency for s in self.served]) if self.served else np.zeros(1)
        n_scen = sum(s.n_scen for s in self.served)
        n_ok = sum(s.n_converged for s in self.served)
        worst = max((s.max_mismatch for s in self.served), default=0.0)
        per_net = {}
        for s in self.served:
            d = per_net.setdefault(s.network, {"requests": 0, "scenarios": 0, "lat": []})
            d["requests"] += 1
            d["scenarios"] += s.n_scen
            d["lat"].append(s.latency)
        nets = {k: {"requests": v["requests"], "scenarios": v["scenarios"],
                    "p50_ms": float(np.percentile(v["lat"], 50) * 1e3),
                    "p99_ms": float(np.percentile(v["lat"], 99) * 1e3)} for k, v in sorted(per_net.items())}
        return {
            "requests": len(self.served),
            "failed_requests": len(self.failed),
            "scenarios": n_scen,
            "converged": n_ok,
            "max_converged_mismatch": worst,
            "duration_s": self.duration,
            "solves_per_s": n_ok / self.duration if self.duration > 0 else 0.0,
            "offered_scen_per_s": n_scen / self.offered_span if self.offered_span > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "max_ms": float(lat.max() * 1e3),
            "mean_submit_lag_ms": float(np.mean([s.submit_lag for s in self.served]) * 1e3) if self.served else 0.0,
            # the parts of the latency, each at its own 50th and 99th percentile
            "parts_ms": {k: {"p50": float(np.percentile(x, 50) * 1e3), "p99": float(np.percentile(x, 99) * 1e3)}
                         for k, x in (("submit_lag", [s.submit_lag for s in self.served] or [0.0]),
                                      ("queue", [s.queue for s in self.served] or [0.0]),
                                      ("service", [s.service for s in self.served] or [0.0]))},
            "per_network": nets,
            "tol": tol,
        }


def replay(engines, trace, inputs, *, tol: float = 1e-8, speed: float = 1.0,
           timeout_s: float = 120.0, switch_interval: float = 2e-4, pause_gc: bool = True) -> ReplayStats:
    """Play ``trace`` (requests with rid, t_arrive, network, n_scen) against ``engines``.

    ``inputs(req)`` returns the request's input arrays (host).  ``speed`` > 1
    compresses the arrival times.  Requests still unfinished ``timeout_s``
    after the last arrival are reported as failed.  One thread submits each
    request when its arrival time comes; a second thread harvests finished
    requests (poll, fetch, accounting), so fetching large results never
    delays a submission.  While the trace plays, the interpreter's thread
    switch interval is ``switch_interval`` seconds (Python's default is 5
    ms, which a sleeping submitter could otherwise wait for while the
    harvester runs Python code), and with ``pause_gc`` the cyclic garbage
    collector is off (one collection before; a full collection in a large
    process holds the interpreter for tens of milliseconds, which would
    stall both threads and show up as latency of every engine).
    """
    order = sorted(trace, key=lambda r: r.t_arrive)
    pending: dict[tuple[int, int], tuple] = {}
    stats = ReplayStats()
    if not order:
        return stats
    staged = [(r, inputs(r)) for r in order]
    lock = threading.Lock()
    submitted_all = threading.Event()
    gc_was = gc.isenabled()
    if pause_gc:
        gc.collect()
        gc.disable()
    t0 = time.perf_counter()

    def harvest_once(wait: float) -> bool:
        got = False
        for k, eng in enumerate(engines):
            for rid in eng.poll(256, wait if not got and k == 0 else 0.0):
                got = True
                with lock:
                    req, t_sub_host = pending.pop((k, rid))
                try:
                    res = eng.fetch(rid)
                except Exception as e:   # a failed launch fails only its own requests
                    with lock:
                        stats.failed.append((rid, str(e)))
                    continue
                ok = res.converged.astype(bool) & (res.mismatch <= tol)
                sub, launch, done = (float(x) for x in res.times)
                s = Served(rid=rid, network=req.network, n_scen=req.n_scen, t_arrive=req.t_arrive,
                           submit_lag=t_sub_host - req.t_arrive / speed, queue=launch - sub,
                           service=done - launch, n_converged=int(ok.sum()),
                           max_mismatch=float(res.mismatch[ok].max()) if ok.any() else float("nan"))
                s.t_done = req.t_arrive / speed + s.latency
                with lock:
                    stats.served.append(s)
        return got

    def harvester() -> None:
        deadline = None
        while True:
            with lock:
                left = len(pending)
            if submitted_all.is_set():
                if left == 0:
                    return
                if deadline is None:
                    deadline = time.perf_counter() + timeout_s
                elif time.perf_counter() > deadline:
                    return
            harvest_once(0.001)

    def play() -> None:
        th = threading.Thread(target=harvester, daemon=True)
        th.start()
        for req, arrays in staged:
            ahead = req.t_arrive / speed - (time.perf_counter() - t0)
            if ahead > 0:
                time.sleep(ahead)   # releases the interpreter lock to the harvester
            eng = engines[req.network]
            with lock:
                pending[(req.network, req.rid)] = (req, time.perf_counter() - t0)
            try:
                eng.submit(req.rid, *arrays)
            except Exception as e:     # e.g. a request larger than the engine's slots
                with lock:
                    pending.pop((req.network, req.rid))
                    stats.failed.append((req.rid, str(e)))
        submitted_all.set()
        th.join()

    old_switch = sys.getswitchinterval()
    sys.setswitchinterval(switch_interval)
    try:
        play()
    finally:
        sys.setswitchinterval(old_switch)
        if pause_gc and gc_was:
            gc.enable()
    with lock:
        for (k, rid), _ in pending.items():
            stats.failed.append((rid, "not finished before the time-out"))
    t_first = order[0].t_arrive / speed
    stats.duration = max((s.t_done for s in stats.served), default=t_first) - t_first
    stats.offered_span = (order[-1].t_arrive - order[0].t_arrive) / speed
    return stats
