"""Benchmark: converged power-flow solves per second on one MI355X.

Default workload (one JSON line on stdout): batched Newton-Raphson on the
synthetic 2000-bus meshed grid (1 slack, 300 PV, 1699 PQ, 2600 branches) with a
batch of 1024 scenarios (+/-20% per-bus load and generation multipliers), flat
start, converged at max |mismatch| <= 1e-8 pu, FP64.  One "step" is one batched
solve of all 1024 scenarios (one kernel launch).  The same line carries the
mixed-precision run (FP32 GMRES inside FP64 mismatch and update), per-step
latency percentiles, the roofline of the solve kernel and the CPU oracle's rate.

Other workloads (--workload): tx30 (30-bus, batch 64), feeder (300-bus / 900-node
feeder Z-bus, batch 4096), adjoint (2000-bus, batch 256), serving (Poisson mix).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_MFMA_TFLOPS = 78.6
FP32_MFMA_TFLOPS = 157.3
METRIC = "converged PF solves/sec @<=1e-8 pu mismatch, FP64 vs mixed; p50/p99 latency"


# ------------------------------------------------------------------ CPU oracle
# Forked workers inherit numpy's BLAS thread pool as it was started in the
# parent, so the thread count is capped through threadpoolctl (environment
# variables set after numpy is loaded have no effect).
def _oracle_tx_chunk(args):
    cfg_name, cols = args
    from threadpoolctl import threadpool_limits
    from oracle import nr
    from workloads import transmission as tx
    cfg = getattr(tx, cfg_name)
    g = tx.make_grid(cfg)
    b = tx.make_batch(g, cfg)
    with threadpool_limits(1):
        t = time.perf_counter()
        _, _, ok, _ = nr.nr_solve_batch(g, b, columns=np.asarray(cols))
        return int(ok.sum()), time.perf_counter() - t


def _oracle_feeder_chunk(args):
    cols, = args
    from threadpoolctl import threadpool_limits
    from oracle import zbus
    from workloads import feeder as fdm
    cfg = fdm.FEEDER300
    fd = fdm.make_feeder(cfg)
    b = fdm.make_batch(fd, cfg)
    sub = fdm.FeederBatch(b.s_wye[cols], b.s_delta[cols])
    with threadpool_limits(1):
        setup = zbus.zbus(fd)   # set-up is excluded from the timing, as on the GPU side
        t = time.perf_counter()
        res = zbus.zbus_solve(fd, sub, setup=setup)
        return int(res.converged.sum()), time.perf_counter() - t


def _oracle_feeder_batched(args):
    """The feeder oracle on one batch with the host's BLAS threads: the batched
    product Z @ I over all scenarios at once, the strongest plain-CPU form."""
    cols, threads = args
    from threadpoolctl import threadpool_limits
    from oracle import zbus
    from workloads import feeder as fdm
    cfg = fdm.FEEDER300
    fd = fdm.make_feeder(cfg)
    b = fdm.make_batch(fd, cfg)
    sub = fdm.FeederBatch(b.s_wye[cols], b.s_delta[cols])
    with threadpool_limits(threads):
        setup = zbus.zbus(fd)
        t = time.perf_counter()
        res = zbus.zbus_solve(fd, sub, setup=setup)
        return int(res.converged.sum()), time.perf_counter() - t


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _pool_leg(kind: str, n_samples: int, workers: int) -> dict:
    """One leg: n_samples scenarios split over `workers` processes, one core
    and one BLAS thread each; the rate uses the slowest worker's solve time."""
    cols = np.arange(n_samples)
    chunks = [c.tolist() for c in np.array_split(cols, workers) if len(c)]
    ctxm = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctxm.Pool(len(chunks)) as pool:
        if kind == "feeder":
            out = pool.map(_oracle_feeder_chunk, [(c,) for c in chunks])
        else:
            out = pool.map(_oracle_tx_chunk, [(kind, c) for c in chunks])
    wall = time.perf_counter() - t0
    solved = sum(o[0] for o in out)
    busy = max(o[1] for o in out)
    return {"workers": len(chunks), "scenarios": n_samples, "converged": solved, "value": solved / busy,
            "slowest_worker_s": busy, "pool_wall_s": wall, "cpu_seconds": float(sum(o[1] for o in out))}


def cpu_baseline(kind: str, n_samples: int, workers: int) -> dict:
    """Time the oracle on bounded samples of the workload's batch: a 1-core
    per-scenario loop, then worker pools of 8, 16 and all usable cores (one
    core and one BLAS thread per worker, the paper's 1/8/16-worker CPU
    baselines), and for the feeder also the batched Z @ I product with all
    cores' BLAS.  The headline value is the largest pool's rate.

    Runs before the GPU is touched (fork start method)."""
    nproc = os.cpu_count() or 1
    per_worker = max(1, n_samples // max(1, workers))
    legs = [_pool_leg(kind, max(4, per_worker), 1)]
    for w in sorted({min(8, workers), min(16, workers), workers}):
        if w > 1:
            legs.append(_pool_leg(kind, per_worker * w, w))
    if kind == "feeder":
        ctxm = mp.get_context("fork")
        with ctxm.Pool(1) as pool:
            solved, busy = pool.map(_oracle_feeder_batched, [(list(range(n_samples)), workers)])[0]
        legs.append({"workers": 1, "blas_threads": workers, "scenarios": n_samples, "converged": solved,
                     "value": solved / busy, "solve_s": busy, "form": "batched Z @ I, all-core BLAS"})
    main = max((g for g in legs if "blas_threads" not in g), key=lambda g: g["workers"])
    return {"value": main["value"], "unit": "solves/s", "cores": main["workers"], "kind": "oracle",
            "sample": f"{main['scenarios']} scenarios of the same batch, {main['workers']} worker processes "
                      f"(one core each, BLAS 1 thread), slowest worker's solve time "
                      f"{main['slowest_worker_s']:.2f} s (pool wall {main['pool_wall_s']:.2f} s incl. start-up)",
            "cpu_seconds": main["cpu_seconds"], "nproc": nproc, "cpu_model": _cpu_model(), "legs": legs}


# ------------------------------------------------------------------ GPU timing
def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_steps(fn, steps: int, warmup: int):
    """Run fn() warmup + steps times; returns per-step ms from HIP events on the
    current stream (each step's event pair brackets exactly its launches)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    pairs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        a, b = _events()
        a.record()
        out = fn()
        b.record()
        pairs.append((a, b))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([a.elapsed_time(b) for a, b in pairs])
    return ms, wall, out


_CSRC = "paper_2605_14103_amd/csrc/"
# Sources whose change invalidates a committed counter summary, per kernel family.
TRAFFIC_SOURCES = {
    "nr": tuple(_CSRC + f for f in ("nr_kernels.hip", "device_ops.hpp", "tx.hpp", "tx_network.cpp", "factor.cpp",
                                    "sell.hpp", "sell.cpp", "api.cpp", "api_tx.cpp")),
    "zbus": tuple(_CSRC + f for f in ("zbus_kernels.hip", "device_ops.hpp", "dist.hpp", "dist_network.cpp",
                                      "zfactor.hpp", "zfactor.cpp", "sell.hpp", "sell.cpp", "api.cpp",
                                      "api_dist.cpp")),
}


def source_digest(family: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES[family]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(profile: str, key: str, family: str = "nr") -> float | None:
    """HBM bytes per launch from a committed counter summary, or None when the
    kernel sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("TRAFFIC_JSON "):
            rec = json.loads(line[len("TRAFFIC_JSON "):])
    if rec is None or source_digest(family) != rec.get("source_sha256_16"):
        return None
    return rec.get(key)


def bench_tx(cfg_name: str, steps: int, warmup: int, cpu: dict | None, block_jacobi: int = 0,
             direct: bool = True) -> dict:
    import torch

    from paper_2605_14103_amd import pf
    from workloads import transmission as tx
    cfg = getattr(tx, cfg_name)
    grid = tx.make_grid(cfg)
    batch = tx.make_batch(grid, cfg)
    ctx = pf.Context(0)
    net = pf.TxNetwork.from_grid(ctx, grid)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    p, q, vm = dev(batch.p_inj), dev(batch.q_inj), dev(batch.vm_set)
    B = batch.batch
    runs = {}
    for prec in ("fp64", "mixed"):
        out = net.solve(p, q, vm, precision=pf.precision(prec))
        ms, wall, out = time_steps(lambda: net.solve(p, q, vm, out=out, precision=pf.precision(prec)), steps, warmup)
        conv = int(out.converged.sum().item())
        mean_ms = float(ms.mean())
        work = float(out.work_bytes.sum().item())
        runs[prec] = {
            "value": conv / (mean_ms * 1e-3), "ms_per_step": mean_ms, "wall_s": wall,
            "converged": conv, "batch": B,
            "latency_ms": {"p50": float(np.percentile(ms, 50)), "p99": float(np.percentile(ms, 99))},
            "newton_iters_mean": float(out.newton_iters.double().mean().item()),
            "gmres_iters_mean": float(out.gmres_iters.double().mean().item()),
            "max_mismatch": float(out.mismatch.max().item()),
            "algorithmic_bytes_per_launch": work,
            "achieved_GBs": work / (mean_ms * 1e-3) / 1e9,
        }
    if block_jacobi:
        # the block-Jacobi reading of the preconditioner (diagonal blocks of 32
        # buses) against the exact (B' + eps I)^-1, (B'' + eps I)^-1 default
        net_bj = pf.TxNetwork.from_grid(ctx, grid, precond_block=block_jacobi)
        for prec in ("fp64", "mixed"):
            out = net_bj.solve(p, q, vm, precision=pf.precision(prec))
            ms, wall, out = time_steps(lambda: net_bj.solve(p, q, vm, out=out, precision=pf.precision(prec)),
                                       steps, warmup)
            conv = int(out.converged.sum().item())
            mean_ms = float(ms.mean())
            runs[f"{prec}_block_jacobi{block_jacobi}"] = {
                "value": conv / (mean_ms * 1e-3), "ms_per_step": mean_ms, "converged": conv, "batch": B,
                "newton_iters_mean": float(out.newton_iters.double().mean().item()),
                "gmres_iters_mean": float(out.gmres_iters.double().mean().item()),
                "max_mismatch": float(out.mismatch.max().item()),
                "achieved_GBs": float(out.work_bytes.sum().item()) / (mean_ms * 1e-3) / 1e9}
            print(f"[bench] {cfg_name} block-Jacobi({block_jacobi}) {prec}: {mean_ms:.3f} ms, "
                  f"{conv} converged", file=sys.stderr, flush=True)
        net_bj.close()
    if direct and grid.n_bus <= 2048:
        # the direct Newton step (per-scenario sparse LU, FP64) on the same batch
        out = net.solve(p, q, vm, nr_direct=1)
        ms, wall, out = time_steps(lambda: net.solve(p, q, vm, out=out, nr_direct=1), steps, warmup)
        conv = int(out.converged.sum().item())
        runs["fp64_direct"] = {
            "value": conv / (float(ms.mean()) * 1e-3), "ms_per_step": float(ms.mean()), "converged": conv,
            "latency_ms": {"p50": float(np.percentile(ms, 50)), "p99": float(np.percentile(ms, 99))},
            "newton_iters_mean": float(out.newton_iters.double().mean().item())}
    # spot parity against the oracle (the rate counts only converged solves)
    from oracle import nr as onr
    cols = np.array([0, B - 1])
    V, _, ok, _ = onr.nr_solve_batch(grid, batch, columns=cols)
    for prec in ("fp64", "mixed"):
        res = net.solve(p, q, vm, precision=pf.precision(prec))
        torch.cuda.synchronize()
        v = res.v.cpu().numpy()[cols]
        runs[prec]["max_abs_V_err_vs_oracle"] = float(np.abs(np.abs(v) - np.abs(V)).max())
        runs[prec]["max_angle_err_vs_oracle"] = float(np.abs(np.angle(v * np.conj(V))).max())
    r = runs["fp64"]
    line = {
        "metric": METRIC, "value": r["value"], "unit": "solves/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{cfg_name}: NR-GMRES(30) left-preconditioned by the exact (B'+eps I)^-1, "
                               f"(B''+eps I)^-1 of eqs. (8)-(9), {grid.n_bus} buses, batch {B}, flat start, "
                               f"tol 1e-8",
                   "global_batch": B, "n_bus": grid.n_bus, "branches": grid.n_branch,
                   "parallelism": "one workgroup per scenario"},
        "latency_ms": r["latency_ms"],
        "roofline": {"bound": "hbm", "achieved": r["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": r["achieved_GBs"] / HBM_PEAK_GBS,
                     "traffic": (measured_traffic(f"nr_kernel_{cfg_name.lower()}_b{B}.txt", "fp64")
                                 if cfg_name == "TX2000" else None),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": "nr_kernel<double, 256, 8>" if grid.n_bus == 2000 else "nr_kernel<double>",
                     "bytes_per_launch": r["algorithmic_bytes_per_launch"]},
        "fp64": runs["fp64"], "mixed": runs["mixed"],
        "mixed_vs_fp64": runs["mixed"]["value"] / r["value"],
        "direct": runs.get("fp64_direct"),
        "block_jacobi": ({k: v for k, v in runs.items() if "block_jacobi" in k} or None),
        "network": net.info,
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    net.close()
    ctx.close()
    return line


def bench_feeder(steps: int, warmup: int, cpu: dict | None) -> dict:
    import torch

    from paper_2605_14103_amd import pf
    from workloads import feeder as fdm
    cfg = fdm.FEEDER300
    fd = fdm.make_feeder(cfg)
    batch = fdm.make_batch(fd, cfg)
    ctx = pf.Context(0)
    net = pf.DistNetwork.from_feeder(ctx, fd)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    sw, sd = dev(batch.s_wye), dev(batch.s_delta)
    B = batch.batch
    nN = net.info["n_free"]
    runs = {}
    for prec, sparse, asy in (("fp64", 0, 0), ("mixed", 0, 0), ("fp64", 1, 0), ("mixed", 1, 0), ("fp64", 0, 1),
                              ("mixed", 0, 1)):
        key = prec + ("_sparse" if sparse else "") + ("_async" if asy else "")
        ms, wall, out = time_steps(
            lambda: net.solve(sw, sd, precision=pf.precision(prec), zbus_sparse=sparse, zbus_async=asy),
            steps, warmup)
        conv = int(out.converged.sum().item())
        its = out.iters.double()
        gemm_flops = 8.0 * nN * nN * float(its.sum().item())
        mean_ms = float(ms.mean())
        runs[key] = {"value": conv / (mean_ms * 1e-3), "ms_per_step": mean_ms, "converged": conv,
                     "iters_mean": float(its.mean().item()), "max_mismatch": float(out.mismatch.max().item()),
                     "latency_ms": {"p50": float(np.percentile(ms, 50)), "p99": float(np.percentile(ms, 99))}}
        if not sparse:
            runs[key]["useful_gemm_TFLOPs"] = gemm_flops / (mean_ms * 1e-3) / 1e12
    r = runs["fp64"]
    tf = r["useful_gemm_TFLOPs"]
    line = {"metric": METRIC, "value": r["value"], "unit": "solves/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"feeder300: Z-bus, {fd.n_node} phase nodes, batch {B}", "global_batch": B},
            "latency_ms": r["latency_ms"],
            "roofline": {"bound": "mfma", "achieved": tf, "peak": FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                         "frac": tf / FP64_MFMA_TFLOPS,
                         "traffic": measured_traffic("zbus_feeder300_b4096.txt", "gemm_fp64", "zbus"),
                         "traffic_unit": "HBM bytes per full zb_gemm_direct<double> launch (rocprofv3 FETCH_SIZE + "
                                         "WRITE_SIZE, copy-calibrated)",
                         "kernel": "zb_gemm_direct<double>",
                         "basis": "useful complex flops (8 nN^2 per scenario and iteration) over the whole "
                                  "solve time, residual kernels and launch gaps included"},
            "fp64": runs["fp64"], "mixed": runs["mixed"],
            "sparse_variant": {"fp64": runs["fp64_sparse"], "mixed": runs["mixed_sparse"]},
            "async_enqueue": {"fp64": runs["fp64_async"], "mixed": runs["mixed_async"]},
            "mixed_vs_fp64": runs["mixed"]["value"] / r["value"]}
    if cpu is not None:
        line["cpu_baseline"] = cpu
    net.close()
    ctx.close()
    return line


def bench_tx_switch(steps: int, warmup: int) -> dict:
    """Topology-action batch on the 2000-bus grid: batch 1024, every scenario
    with one branch out of service (its own Ybus values on the shared pattern),
    against the same loads with the network's own values."""
    import torch

    from paper_2605_14103_amd import pf
    from workloads import transmission as tx
    cfg = tx.TX2000
    grid = tx.make_grid(cfg)
    batch = tx.make_batch(grid, cfg)
    on = tx.make_outages(grid, batch.batch, n_out=1, seed=cfg.seed + 7)
    ctx = pf.Context(0)
    net = pf.TxNetwork.from_grid(ctx, grid)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    p, q, vm = dev(batch.p_inj), dev(batch.q_inj), dev(batch.vm_set)
    yv = dev(net.ybus_switch(on))
    B = batch.batch
    runs = {}
    # Two of these outages leave no solution near flat start (the oracle fails on
    # them as well); with the default max_newton = 20 those two scenarios set the
    # batch time, so the run capped at 8 Newton steps (every converging scenario
    # here needs at most 7) is reported beside it.
    for prec in ("fp64", "mixed"):
        for kind in ("shared", "switch", "switch_max_newton8"):
            if kind == "shared":
                fn = lambda: net.solve(p, q, vm, precision=pf.precision(prec))  # noqa: E731
            elif kind == "switch":
                fn = lambda: net.solve_yvals(p, q, vm, yv, precision=pf.precision(prec))  # noqa: E731
            else:
                fn = lambda: net.solve_yvals(p, q, vm, yv, precision=pf.precision(prec), max_newton=8)  # noqa: E731
            ms, _, out = time_steps(fn, steps, warmup)
            conv = int(out.converged.sum().item())
            mean_ms = float(ms.mean())
            runs[f"{prec}_{kind}"] = {
                "value": conv / (mean_ms * 1e-3), "ms_per_step": mean_ms, "converged": conv,
                "newton_iters_mean": float(out.newton_iters.double().mean().item()),
                "gmres_iters_mean": float(out.gmres_iters.double().mean().item()),
                "algorithmic_bytes_per_launch": float(out.work_bytes.sum().item()),
                "achieved_GBs": float(out.work_bytes.sum().item()) / (mean_ms * 1e-3) / 1e9}
            print(f"[switch] {prec} {kind} {mean_ms:.3f} ms, {conv} converged, "
                  f"gmres {runs[f'{prec}_{kind}']['gmres_iters_mean']:.1f}", file=sys.stderr, flush=True)
    r = runs["fp64_switch_max_newton8"]
    net.close()
    ctx.close()
    return {"metric": METRIC, "value": r["value"], "unit": "solves/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"tx2000 N-1 actions: one branch out per scenario, batch {B}, "
                                   "max_newton 8", "global_batch": B},
            "runs": runs}


def bench_direct_sizes(steps: int, warmup: int) -> dict:
    """Newton linear solver against grid size: preconditioned GMRES (FP64 and
    mixed) against the direct step (per-scenario sparse LU, FP64), batch 64
    and 1024, grids of 30 to 500 buses."""
    import torch

    from paper_2605_14103_amd import pf
    from workloads import transmission as tx
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    rows = []
    ctx = pf.Context(0)
    for n_bus in (30, 118, 300, 500):
        cfg = tx.TX30 if n_bus == 30 else tx.TxConfig(
            f"tx{n_bus}", n_bus=n_bus, n_pv=max(5, n_bus * 15 // 100), n_branch=int(n_bus * 1.3), batch=64,
            seed=n_bus, perturbation="uniform", spread=0.2)
        grid = tx.make_grid(cfg)
        net = pf.TxNetwork.from_grid(ctx, grid)
        for B in (64, 1024):
            batch = tx.make_batch(grid, cfg, batch=B)
            p, q, vm = dev(batch.p_inj), dev(batch.q_inj), dev(batch.vm_set)
            for kind, opts in (("gmres_fp64", {}), ("gmres_mixed", {"precision": pf.precision("mixed")}),
                               ("direct", {"nr_direct": 1})):
                out = net.solve(p, q, vm, **opts)
                ms, _, out = time_steps(lambda: net.solve(p, q, vm, out=out, **opts), steps, warmup)
                conv = int(out.converged.sum().item())
                rows.append({"n_bus": n_bus, "batch": B, "solver": kind, "ms": float(ms.mean()),
                             "solves_per_s": conv / (float(ms.mean()) * 1e-3), "converged": conv,
                             "newton_iters_mean": float(out.newton_iters.double().mean().item())})
                print(f"[direct] tx{n_bus} B={B} {kind} {ms.mean():.3f} ms", file=sys.stderr, flush=True)
        net.close()
    ctx.close()
    best = max(r["solves_per_s"] for r in rows if r["n_bus"] == 30)
    return {"metric": METRIC, "value": best, "unit": "solves/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "Newton linear solver sweep: GMRES against the direct step, 30-500 buses"},
            "sizes": rows}


def bench_feeder_sizes(steps: int, warmup: int) -> dict:
    """Dense Z product against the sparse Y_NN factor as the feeder grows (batch 1024, both precisions)."""
    import torch

    from paper_2605_14103_amd import pf
    from workloads import feeder as fdm
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    rows = []
    ctx = pf.Context(0)
    for n_bus in (100, 300, 600, 908):
        cfg = fdm.FeederConfig(f"feeder{n_bus}", n_bus=n_bus, max_depth=25, batch=1024, seed=n_bus)
        fd = fdm.make_feeder(cfg)
        batch = fdm.make_batch(fd, cfg)
        t0 = time.perf_counter()
        net = pf.DistNetwork.from_feeder(ctx, fd)
        setup_s = time.perf_counter() - t0
        sw, sd = dev(batch.s_wye), dev(batch.s_delta)
        for sparse in (0, 1):
            for prec in ("fp64", "mixed"):
                ms, _, out = time_steps(
                    lambda: net.solve(sw, sd, precision=pf.precision(prec), zbus_sparse=sparse), steps, warmup)
                conv = int(out.converged.sum().item())
                rows.append({"workload": cfg.name, "free_nodes": net.info["n_free"], "batch": cfg.batch,
                             "update": "sparse" if sparse else "dense", "precision": prec,
                             "ms": float(ms.mean()), "solves_per_s": conv / (float(ms.mean()) * 1e-3),
                             "converged": conv, "iters_mean": float(out.iters.double().mean().item()),
                             "setup_s": setup_s})
                print(f"[sizes] {cfg.name} nN={net.info['n_free']} {rows[-1]['update']} {prec} "
                      f"{ms.mean():.3f} ms", file=sys.stderr, flush=True)
        net.close()
    ctx.close()
    best = max(r["solves_per_s"] for r in rows if r["workload"] == "feeder300" and r["precision"] == "fp64")
    return {"metric": METRIC, "value": best, "unit": "solves/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "feeder size sweep: 100-908 buses, batch 1024, dense Z against sparse Y_NN"},
            "sizes": rows}


def bench_adjoint(steps: int, warmup: int) -> dict:
    """Branch-loss gradient w.r.t. PQ injections (adjoint GMRES) on the 2000-bus grid, batch 256."""
    import torch

    from paper_2605_14103_amd import pf
    from workloads import transmission as tx
    cfg = tx.TX2000_ADJ
    grid = tx.make_grid(cfg)
    batch = tx.make_batch(grid, cfg)
    ctx = pf.Context(0)
    net = pf.TxNetwork.from_grid(ctx, grid)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    p, q, vm = dev(batch.p_inj), dev(batch.q_inj), dev(batch.vm_set)
    B = batch.batch
    res = net.solve(p, q, vm)
    loss, g = net.branch_loss(res.v)

    def step():
        l, gv = net.branch_loss(res.v)
        return net.adjoint(res.v, gv)

    ms, wall, out = time_steps(step, steps, warmup)
    ok = int(out[3].sum().item())
    mean_ms = float(ms.mean())
    line = {"metric": "adjoint gradients/s (branch loss w.r.t. PQ injections)", "value": ok / (mean_ms * 1e-3),
            "unit": "gradients/s", "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": mean_ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"tx2000_adj: loss + transposed-Jacobian GMRES, batch {B}", "global_batch": B},
            "adjoint_gmres_iters_mean": float(out[2].double().mean().item()),
            "latency_ms": {"p50": float(np.percentile(ms, 50)), "p99": float(np.percentile(ms, 99))}}
    net.close()
    ctx.close()
    return line


def bench_serving(n_requests: int, lam: float, streams=(1, 3, 1), step_iters=(20, 1, 2), half: bool = True,
                  forcing: int = 0, feeder_sparse: int = 0) -> dict:
    """Replay the Poisson serving mix (30-bus grid, 2000-bus grid, 900-node feeder).

    streams and step_iters are per engine (30-bus, 2000-bus, feeder);
    feeder_sparse = 1 runs the feeder engine's update by the sparse factor of
    Y_NN instead of the dense Z product."""
    from paper_2605_14103_amd import pf, serve
    from workloads import feeder as fdm
    from workloads import serving as wsv
    from workloads import transmission as tx
    g30 = tx.make_grid(tx.TX30)
    g2k = tx.make_grid(tx.TX2000)
    fd = fdm.make_feeder(fdm.FEEDER300)
    trace = wsv.make_trace(wsv.SERVING, n_requests=n_requests, lam=lam)

    def inputs(r):
        if r.network == 0:
            b = tx.make_batch(g30, tx.TX30, batch=r.n_scen, seed=r.seed)
            return b.p_inj, b.q_inj, b.vm_set
        if r.network == 1:
            b = tx.make_batch(g2k, tx.TX2000, batch=r.n_scen, seed=r.seed)
            return b.p_inj, b.q_inj, b.vm_set
        b = fdm.make_batch(fd, fdm.FEEDER300, batch=r.n_scen, seed=r.seed)
        return b.s_wye, b.s_delta

    out = {}
    half_trace = wsv.make_trace(wsv.SERVING, n_requests=n_requests // 2, lam=lam / 2)
    runs = [("fp64", trace, "fp64"), ("mixed", trace, "mixed")]
    if half:
        runs.append(("fp64", half_trace, "fp64_half_load"))
    for prec, tr, key in runs:
        ctx = pf.Context(0)
        nets = [pf.TxNetwork.from_grid(ctx, g30), pf.TxNetwork.from_grid(ctx, g2k),
                pf.DistNetwork.from_feeder(ctx, fd)]
        budgets = (1 << 30, 24 << 30, 4 << 30)
        extra = ({}, {}, {"zbus_sparse": feeder_sparse})
        engines = [pf.Engine(n, hbm_bytes=b, n_streams=s, precision=pf.precision(prec), step_iters=k,
                             forcing=forcing, **x)
                   for n, b, s, k, x in zip(nets, budgets, streams, step_iters, extra)]
        # warm-up: one small request per engine (code objects, first launches)
        warm = [r for r in wsv.make_trace(wsv.SERVING, n_requests=30, lam=lam) if r.n_scen <= 8][:6]
        serve.replay(engines, warm, inputs, speed=100.0)
        t = time.perf_counter()
        st = serve.replay(engines, tr, inputs)
        summ = st.summary()
        summ["wall_s"] = time.perf_counter() - t
        summ["engines"] = [e.info() for e in engines]
        summ["lambda_per_s"] = lam / 2 if key.endswith("half_load") else lam
        out[key] = summ
        print(f"[serving {key}] {summ['requests']} requests, {summ['solves_per_s']:.0f} solves/s, "
              f"p50 {summ['p50_ms']:.2f} ms, p99 {summ['p99_ms']:.2f} ms", file=sys.stderr, flush=True)
        for e in engines:
            e.close()
        for n in nets:
            n.close()
        ctx.close()
    r = out["fp64"]
    return {"metric": METRIC, "value": r["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": 1,
            "warmup": 1, "ms_per_step": r["duration_s"] * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": f"serving mix: Poisson lambda={lam}/s, {n_requests} requests over tx30, "
                                   f"tx2000 and feeder300, 1-512 scenarios each, tol 1e-8",
                       "streams": list(streams), "step_iters": list(step_iters), "forcing": forcing,
                       "feeder_update": "sparse Y_NN factor" if feeder_sparse else "dense Z product"},
            "latency_ms": {"p50": r["p50_ms"], "p99": r["p99_ms"]},
            "fp64": out["fp64"], "mixed": out["mixed"], "fp64_half_load": out.get("fp64_half_load")}


def bench_sweep(steps: int, warmup: int) -> dict:
    """Solve time against batch size (2000-bus grid and 900-node feeder, both precisions)."""
    import torch

    from paper_2605_14103_amd import pf
    from workloads import feeder as fdm
    from workloads import transmission as tx
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    rows = []
    ctx = pf.Context(0)
    grid = tx.make_grid(tx.TX2000)
    net = pf.TxNetwork.from_grid(ctx, grid)
    for B in (1, 16, 64, 256, 1024, 4096):
        batch = tx.make_batch(grid, tx.TX2000, batch=B)
        p, q, vm = dev(batch.p_inj), dev(batch.q_inj), dev(batch.vm_set)
        for prec in ("fp64", "mixed"):
            out = net.solve(p, q, vm, precision=pf.precision(prec))
            ms, _, out = time_steps(lambda: net.solve(p, q, vm, out=out, precision=pf.precision(prec)), steps, warmup)
            conv = int(out.converged.sum().item())
            rows.append({"workload": "tx2000", "batch": B, "precision": prec, "ms": float(ms.mean()),
                         "solves_per_s": conv / (float(ms.mean()) * 1e-3), "converged": conv})
            print(f"[sweep] tx2000 B={B} {prec} {ms.mean():.3f} ms", file=sys.stderr, flush=True)
    net.close()
    fd = fdm.make_feeder(fdm.FEEDER300)
    dnet = pf.DistNetwork.from_feeder(ctx, fd)
    for B in (1, 16, 64, 256, 1024, 4096, 16384):
        batch = fdm.make_batch(fd, fdm.FEEDER300, batch=B)
        sw, sd = dev(batch.s_wye), dev(batch.s_delta)
        for prec in ("fp64", "mixed"):
            ms, _, out = time_steps(lambda: dnet.solve(sw, sd, precision=pf.precision(prec)), steps, warmup)
            conv = int(out.converged.sum().item())
            rows.append({"workload": "feeder300", "batch": B, "precision": prec, "ms": float(ms.mean()),
                         "solves_per_s": conv / (float(ms.mean()) * 1e-3), "converged": conv})
            print(f"[sweep] feeder300 B={B} {prec} {ms.mean():.3f} ms", file=sys.stderr, flush=True)
    dnet.close()
    ctx.close()
    best = max(r["solves_per_s"] for r in rows if r["workload"] == "tx2000" and r["precision"] == "fp64")
    return {"metric": METRIC, "value": best, "unit": "solves/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic", "config": {"workload": "batch sweep: tx2000 B=1..4096, feeder300 B=1..16384"},
            "sweep": rows}


def counters_run(workload: str) -> dict:
    """One launch per precision, plus a calibration copy, for hardware-counter runs.

    Run under `rocprofv3 --pmc FETCH_SIZE` (then WRITE_SIZE) to measure HBM
    traffic per launch; the calibration is one device-to-device copy of
    512 MiB (read 512 MiB, write 512 MiB) whose counter values give the scale
    of the counters.  Prints the algorithmic bytes of each launch.
    """
    import torch

    from paper_2605_14103_amd import pf
    n = 64 * 1024 * 1024
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    out = {"calibration_copy_bytes": 8 * n}
    ctx = pf.Context(0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    if workload == "feeder":
        from workloads import feeder as fdm
        fd = fdm.make_feeder(fdm.FEEDER300)
        batch = fdm.make_batch(fd, fdm.FEEDER300)
        net = pf.DistNetwork.from_feeder(ctx, fd)
        sw, sd = dev(batch.s_wye), dev(batch.s_delta)
        for sparse in (0, 1):
            for prec in ("fp64", "mixed"):
                res = net.solve(sw, sd, precision=pf.precision(prec), zbus_sparse=sparse)
                torch.cuda.synchronize()
                out[prec + ("_sparse" if sparse else "")] = {"iters": res.iters.cpu().numpy().tolist()[:4]}
    else:
        from workloads import transmission as tx
        cfg = {"tx2000": tx.TX2000, "tx30": tx.TX30}[workload]
        grid = tx.make_grid(cfg)
        batch = tx.make_batch(grid, cfg)
        net = pf.TxNetwork.from_grid(ctx, grid)
        p, q, vm = dev(batch.p_inj), dev(batch.q_inj), dev(batch.vm_set)
        for prec in ("fp64", "mixed"):
            res = net.solve(p, q, vm, precision=pf.precision(prec))
            torch.cuda.synchronize()
            out[prec] = {"algorithmic_bytes_per_launch": float(res.work_bytes.sum().item())}
    net.close()
    ctx.close()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tx2000",
                    choices=["tx2000", "tx30", "feeder", "adjoint", "serving", "sweep", "feeder_sizes",
                             "tx2000_switch", "direct_sizes"])
    ap.add_argument("--requests", type=int, default=4000, help="serving: trace length")
    ap.add_argument("--lam", type=float, default=2000.0, help="serving: arrival rate (requests/s)")
    ap.add_argument("--streams", default="1,3,1",
                    help="serving: HIP streams of the 30-bus, 2000-bus and feeder engines")
    ap.add_argument("--step-iters", default="20,1,2",
                    help="serving: Newton updates / fixed-point iterations per engine step, per engine")
    ap.add_argument("--no-half", action="store_true", help="serving: skip the half-load replay")
    ap.add_argument("--forcing", type=int, default=0,
                    help="serving engines: fixed (0, lower tail latency) or adaptive (1) forcing term")
    ap.add_argument("--feeder-update", choices=("sparse", "dense"), default="sparse",
                    help="serving: the feeder engine's update, by the sparse factor of Y_NN (lower latency "
                         "at the small batches a serving step holds) or the dense Z product")
    ap.add_argument("--cpu-samples", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="default workload: the 2000-bus FP64 and mixed solves alone (no block-Jacobi, "
                         "direct-step or other-config runs)")
    ap.add_argument("--counters", action="store_true",
                    help="one launch per precision plus a calibration copy, for rocprofv3 --pmc runs")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {a.gpus}); run with --gpus 1", file=sys.stderr)
        return 2
    if a.counters:
        print(json.dumps(counters_run(a.workload)), flush=True)
        return 0
    workers = min(16, os.cpu_count() or 1)
    cpu = None
    n_samp = {"tx2000": a.cpu_samples, "tx30": 64, "feeder": 512}
    kinds = {"tx2000": "TX2000", "tx30": "TX30", "feeder": "feeder"}
    if not a.no_cpu and a.workload in kinds:
        cpu = cpu_baseline(kinds[a.workload], n_samp[a.workload], workers)
    a.sub_cpu = {}
    if not a.no_cpu and a.workload == "tx2000" and not a.headline_only:
        # the other configs' oracle legs, also before the GPU is touched
        for w in ("tx30", "feeder"):
            a.sub_cpu[w] = cpu_baseline(kinds[w], n_samp[w], workers)
    if a.workload == "feeder":
        line = bench_feeder(a.steps, a.warmup, cpu)
    elif a.workload == "adjoint":
        line = bench_adjoint(a.steps, a.warmup)
    elif a.workload == "serving":
        line = bench_serving(a.requests, a.lam, tuple(int(x) for x in a.streams.split(",")),
                             tuple(int(x) for x in a.step_iters.split(",")), half=not a.no_half, forcing=a.forcing,
                             feeder_sparse=int(a.feeder_update == "sparse"))
    elif a.workload == "sweep":
        line = bench_sweep(a.steps, a.warmup)
    elif a.workload == "feeder_sizes":
        line = bench_feeder_sizes(a.steps, a.warmup)
    elif a.workload == "tx2000_switch":
        line = bench_tx_switch(a.steps, a.warmup)
    elif a.workload == "direct_sizes":
        line = bench_direct_sizes(a.steps, a.warmup)
    elif a.workload == "tx30":
        line = bench_tx("TX30", a.steps, a.warmup, cpu)
    else:
        if a.headline_only:
            line = bench_tx("TX2000", a.steps, a.warmup, cpu, direct=False)
        else:
            line = bench_tx("TX2000", a.steps, a.warmup, cpu, block_jacobi=32)
            line["configs"] = all_configs(a)
    print(json.dumps(line), flush=True)
    return 0


def _sub(line: dict) -> dict:
    """A sub-record: the line without the fields that only the headline carries."""
    return {k: v for k, v in line.items() if k not in ("n_gpus", "scaling", "vs_baseline", "data")}


def all_configs(a) -> dict:
    """The other configurations of the method, each timed as its own line
    would be, so that one default run measures them all: the 30-bus grid
    (batch 64), the 900-node feeder (batch 4096, dense product in FP64 and
    FP32, sparse variant), the adjoint (2000-bus, batch 256) and the serving
    mix at full and half load."""
    out = {}
    for key, fn in (("tx30_b64", lambda: bench_tx("TX30", a.steps, a.warmup, a.sub_cpu.get("tx30"))),
                    ("feeder300_b4096", lambda: bench_feeder(a.steps, a.warmup, a.sub_cpu.get("feeder"))),
                    ("adjoint_tx2000_b256", lambda: bench_adjoint(a.steps, a.warmup)),
                    ("serving_mix", lambda: bench_serving(a.requests, a.lam,
                                                          tuple(int(x) for x in a.streams.split(",")),
                                                          tuple(int(x) for x in a.step_iters.split(",")),
                                                          forcing=a.forcing,
                                                          feeder_sparse=int(a.feeder_update == "sparse")))):
        t = time.perf_counter()
        try:
            out[key] = _sub(fn())
        except Exception as e:  # a failing sub-record must not hide the headline
            out[key] = {"error": f"{type(e).__name__}: {e}"}
        print(f"[bench] {key}: {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    return out


if __name__ == "__main__":
    sys.exit(main())
