"""Python binding of the device library: argument marshalling only.

Every step of the solvers runs in the library's HIP kernels; this module turns
torch tensors (device memory) and numpy arrays (host network data) into the
pointers and sizes of the C ABI in include/pfx.h, and torch's current HIP
stream into the stream argument.

Layout: per-scenario tensors are scenario-major, shape (batch, n) with unit
stride along n; the row stride is passed as ``ld``.  Complex tensors are
complex128 (re, im interleaved, as the ABI expects).
"""
from __future__ import annotations

import ctypes
from ctypes import byref, c_int32, c_void_p
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


def _stream(stream) -> c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


def _dptr(t: torch.Tensor | None) -> c_void_p | None:
    return None if t is None else c_void_p(t.data_ptr())


def _hptr(a: np.ndarray) -> c_void_p:
    return c_void_p(a.ctypes.data)


def _rows(t: torch.Tensor, n: int, dtype: torch.dtype, name: str) -> int:
    """Check a (batch, n) device tensor and return its row stride in elements."""
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != 2 or t.shape[1] != n:
        raise ValueError(f"{name} must have shape (batch, {n}), got {tuple(t.shape)}")
    if t.shape[0] > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} must have unit stride along its second dimension")
    return int(t.stride(0)) if t.shape[0] > 1 else n


def _ld(*pairs) -> int:
    lds = {_rows(t, n, dt, name) for t, n, dt, name in pairs}
    if len(lds) != 1:
        raise ValueError("all per-scenario tensors of one call must share a row stride")
    return lds.pop()


class Context:
    """A device context (one per GPU); owns the networks created in it."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.device = int(device)
        h = c_void_p()
        L.call("pf_context_create", self.device, int(hbm_budget_bytes), byref(h))
        self.h = h

    def bytes(self) -> int:
        return int(L.lib().pf_context_bytes(self.h))

    def close(self) -> None:
        if self.h:
            L.lib().pf_context_destroy(self.h)
            self.h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _setup_opts(setup: dict) -> L.PfOpts:
    return L.opts(**setup)


@dataclass
class TxResult:
    v: torch.Tensor              # complex128 (batch, n_bus)
    newton_iters: torch.Tensor   # int32 (batch,)
    gmres_iters: torch.Tensor    # int32 (batch,)
    converged: torch.Tensor      # uint8 (batch,)
    mismatch: torch.Tensor       # float64 (batch,)
    work_bytes: torch.Tensor | None = None   # float64 (batch,): algorithmic HBM bytes per solve


class TxNetwork:
    """A registered transmission grid (Newton-Raphson, Sec. II-A)."""

    def __init__(self, ctx: Context, n_bus: int, bus_type, f, t, r, x, b, **setup):
        self.ctx = ctx
        self.n_bus = int(n_bus)
        f = np.ascontiguousarray(f, dtype=np.int32)
        t = np.ascontiguousarray(t, dtype=np.int32)
        r = np.ascontiguousarray(r, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        bt = np.ascontiguousarray(bus_type, dtype=np.int8)
        nbr = int(f.shape[0])
        cap = self.n_bus + 2 * nbr
        ptr = np.zeros(self.n_bus + 1, dtype=np.int32)
        col = np.zeros(cap, dtype=np.int32)
        yre = np.zeros(cap)
        yim = np.zeros(cap)
        nnz = c_int32()
        L.call("pf_tx_ybus_from_branches", self.n_bus, nbr, _hptr(f), _hptr(t), _hptr(r), _hptr(x), _hptr(b),
               cap, _hptr(ptr), _hptr(col), _hptr(yre), _hptr(yim), byref(nnz))
        h = c_void_p()
        so = _setup_opts(setup)
        L.call("pf_tx_network_create", ctx.h, self.n_bus, nnz.value, _hptr(ptr), _hptr(col), _hptr(yre),
               _hptr(yim), _hptr(bt), nbr, _hptr(f), _hptr(t), _hptr(r), _hptr(x), _hptr(b), byref(so), byref(h))
        self.h = h
        self.info = self._info()
        k = nnz.value
        self.csr = (ptr, col[:k].copy(), yre[:k].copy(), yim[:k].copy())
        self.branches = (f, t, r, x, b)

    @classmethod
    def from_grid(cls, ctx: Context, grid, **setup) -> "TxNetwork":
        """From a ``workloads.transmission.TxGrid``."""
        return cls(ctx, grid.n_bus, grid.bus_type, grid.f, grid.t, grid.r, grid.x, grid.b, **setup)

    def _info(self) -> dict:
        vals = [c_int32() for _ in range(7)]
        L.call("pf_tx_network_info", self.h, *[byref(v) for v in vals])
        keys = ["n_bus", "n_theta", "n_q", "nnz", "factor_nnz", "core_bp", "core_bpp"]
        return {k: v.value for k, v in zip(keys, vals)}

    def close(self) -> None:
        if self.h:
            L.lib().pf_tx_network_destroy(self.h)
            self.h = c_void_p()

    def _out(self, out: "TxResult | None", B: int, ld: int, dev) -> "TxResult":
        """The caller's output tensors (rows at the input stride) or new ones."""
        n = self.n_bus
        if out is None:
            out = TxResult(v=torch.empty((B, n), dtype=torch.complex128, device=dev),
                           newton_iters=torch.empty(B, dtype=torch.int32, device=dev),
                           gmres_iters=torch.empty(B, dtype=torch.int32, device=dev),
                           converged=torch.empty(B, dtype=torch.uint8, device=dev),
                           mismatch=torch.empty(B, dtype=torch.float64, device=dev),
                           work_bytes=torch.empty(B, dtype=torch.float64, device=dev))
        if B > 1 and out.v.stride(0) != ld:
            raise ValueError("output rows must use the input row stride")
        return out

    def solve(self, p_inj: torch.Tensor, q_inj: torch.Tensor, vm_set: torch.Tensor, *, stream=None,
              out: TxResult | None = None, **opts) -> TxResult:
        """Batched Newton-Raphson from a flat start; see pf_tx_solve."""
        n = self.n_bus
        ld = _ld((p_inj, n, torch.float64, "p_inj"), (q_inj, n, torch.float64, "q_inj"),
                 (vm_set, n, torch.float64, "vm_set"))
        B = int(p_inj.shape[0])
        dev = p_inj.device
        out = self._out(out, B, ld, dev)
        o = L.opts(**opts)
        L.call("pf_tx_solve", self.h, byref(o), B, ld, _dptr(p_inj), _dptr(q_inj), _dptr(vm_set),
               _dptr(out.v), _dptr(out.newton_iters), _dptr(out.gmres_iters), _dptr(out.converged),
               _dptr(out.mismatch), _dptr(out.work_bytes), _stream(stream))
        return out

    def solve_noalloc(self, p_inj: torch.Tensor, q_inj: torch.Tensor, vm_set: torch.Tensor, *,
                      out: TxResult, stream=None, **opts) -> TxResult:
        """As ``solve``, with the library's workspace taken from its fixed device
        array (no device allocation in the call); the caller passes every output
        tensor.  See pf_tx_solve_noalloc."""
        n = self.n_bus
        ld = _ld((p_inj, n, torch.float64, "p_inj"), (q_inj, n, torch.float64, "q_inj"),
                 (vm_set, n, torch.float64, "vm_set"))
        B = int(p_inj.shape[0])
        out = self._out(out, B, ld, p_inj.device)
        o = L.opts(**opts)
        L.call("pf_tx_solve_noalloc", self.h, byref(o), B, ld, _dptr(p_inj), _dptr(q_inj), _dptr(vm_set),
               _dptr(out.v), _dptr(out.newton_iters), _dptr(out.gmres_iters), _dptr(out.converged),
               _dptr(out.mismatch), _dptr(out.work_bytes), _stream(stream))
        return out

    def ybus_switch(self, branch_on: np.ndarray) -> np.ndarray:
        """Per-scenario Ybus values (complex [batch][nnz], this network's CSR
        order) with the branches where ``branch_on`` is 0 switched out; see
        pf_tx_ybus_switch."""
        on = np.ascontiguousarray(branch_on, dtype=np.uint8)
        f, t, r, x, b = self.branches
        if on.ndim != 2 or on.shape[1] != f.shape[0]:
            raise ValueError(f"branch_on must be (batch, {f.shape[0]})")
        ptr, col, yre, yim = self.csr
        nnz = int(col.shape[0])
        out = np.zeros((on.shape[0], nnz), dtype=np.complex128)
        L.call("pf_tx_ybus_switch", self.n_bus, nnz, _hptr(ptr), _hptr(col), _hptr(yre), _hptr(yim),
               int(f.shape[0]), _hptr(f), _hptr(t), _hptr(r), _hptr(x), _hptr(b), int(on.shape[0]), _hptr(on),
               nnz, _hptr(out))
        return out

    def solve_yvals(self, p_inj: torch.Tensor, q_inj: torch.Tensor, vm_set: torch.Tensor, y_vals: torch.Tensor,
                    *, stream=None, out: TxResult | None = None, **opts) -> TxResult:
        """Batched Newton-Raphson with each scenario's own Ybus values (device complex
        [batch][nnz] in this network's CSR order); see pf_tx_solve_yvals."""
        n = self.n_bus
        ld = _ld((p_inj, n, torch.float64, "p_inj"), (q_inj, n, torch.float64, "q_inj"),
                 (vm_set, n, torch.float64, "vm_set"))
        nnz = int(self.csr[1].shape[0])
        B = int(p_inj.shape[0])
        ldy = _ld((y_vals, nnz, torch.complex128, "y_vals"))
        if int(y_vals.shape[0]) != B:
            raise ValueError("y_vals must have one row per scenario")
        dev = p_inj.device
        out = self._out(out, B, ld, dev)
        o = L.opts(**opts)
        L.call("pf_tx_solve_yvals", self.h, byref(o), B, ld, _dptr(p_inj), _dptr(q_inj), _dptr(vm_set),
               ldy, _dptr(y_vals), _dptr(out.v), _dptr(out.newton_iters), _dptr(out.gmres_iters),
               _dptr(out.converged), _dptr(out.mismatch), _dptr(out.work_bytes), _stream(stream))
        return out

    def branch_loss(self, v: torch.Tensor, *, grad: bool = True, stream=None):
        """(loss (batch,), dL/dV in torch's convention or None); see pf_tx_branch_loss."""
        ld = _ld((v, self.n_bus, torch.complex128, "v"))
        B = int(v.shape[0])
        loss = torch.empty(B, dtype=torch.float64, device=v.device)
        g = torch.empty_like(v) if grad else None
        L.call("pf_tx_branch_loss", self.h, B, ld, _dptr(v), _dptr(loss), _dptr(g), _stream(stream))
        return loss, g

    def adjoint(self, v: torch.Tensor, dl_dv: torch.Tensor, *, stream=None, **opts):
        """(grad_p, grad_q, gmres_iters, converged); see pf_tx_adjoint."""
        n = self.n_bus
        ld = _ld((v, n, torch.complex128, "v"), (dl_dv, n, torch.complex128, "dl_dv"))
        B = int(v.shape[0])
        gp = torch.empty((B, n), dtype=torch.float64, device=v.device)
        gq = torch.empty((B, n), dtype=torch.float64, device=v.device)
        if B > 1 and gp.stride(0) != ld:
            gp = torch.empty_strided((B, n), (ld, 1), dtype=torch.float64, device=v.device)
            gq = torch.empty_strided((B, n), (ld, 1), dtype=torch.float64, device=v.device)
        its = torch.empty(B, dtype=torch.int32, device=v.device)
        ok = torch.empty(B, dtype=torch.uint8, device=v.device)
        o = L.opts(**opts)
        L.call("pf_tx_adjoint", self.h, byref(o), B, ld, _dptr(v), _dptr(dl_dv), _dptr(gp), _dptr(gq),
               _dptr(its), _dptr(ok), _stream(stream))
        return gp, gq, its, ok


@dataclass
class DistResult:
    v: torch.Tensor               # complex128 (batch, n_node)
    iters: torch.Tensor           # int32 (batch,)
    converged: torch.Tensor       # uint8 (batch,)
    mismatch: torch.Tensor        # float64 (batch,)
    sum_abs_change: torch.Tensor  # float64 (batch,)


class DistNetwork:
    """A registered three-phase radial feeder (Z-bus fixed point, Sec. II-B)."""

    def __init__(self, ctx: Context, n_bus: int, seg_from, seg_to, z_seg, slack_nodes, v_slack,
                 wye_nodes, delta_nodes, **setup):
        self.ctx = ctx
        self.n_node = 3 * int(n_bus)
        sf = np.ascontiguousarray(seg_from, dtype=np.int32)
        st = np.ascontiguousarray(seg_to, dtype=np.int32)
        z = np.ascontiguousarray(np.asarray(z_seg, dtype=np.complex128))
        nseg = int(sf.shape[0])
        cap = 3 * self.n_node + 18 * nseg   # 3x3 diagonal blocks plus two off-diagonal blocks per segment
        ptr = np.zeros(self.n_node + 1, dtype=np.int32)
        col = np.zeros(cap, dtype=np.int32)
        yre = np.zeros(cap)
        yim = np.zeros(cap)
        nnz = c_int32()
        L.call("pf_dist_ybus_from_segments", int(n_bus), nseg, _hptr(sf), _hptr(st), _hptr(z), cap, _hptr(ptr),
               _hptr(col), _hptr(yre), _hptr(yim), byref(nnz))
        sl = np.ascontiguousarray(slack_nodes, dtype=np.int32)
        vs = np.ascontiguousarray(np.asarray(v_slack, dtype=np.complex128))
        wy = np.ascontiguousarray(wye_nodes, dtype=np.int32)
        de = np.ascontiguousarray(delta_nodes, dtype=np.int32).reshape(-1, 3)
        so = _setup_opts(setup)
        h = c_void_p()
        L.call("pf_dist_network_create", ctx.h, self.n_node, nnz.value, _hptr(ptr), _hptr(col), _hptr(yre),
               _hptr(yim), _hptr(sl), _hptr(vs), int(wy.shape[0]), _hptr(wy), int(de.shape[0]), _hptr(de),
               byref(so), byref(h))
        self.h = h
        vals = [c_int32() for _ in range(4)]
        L.call("pf_dist_network_info", self.h, *[byref(v) for v in vals])
        self.info = dict(zip(["n_node", "n_free", "n_wye", "n_delta"], [v.value for v in vals]))

    @classmethod
    def from_feeder(cls, ctx: Context, fd, **setup) -> "DistNetwork":
        """From a ``workloads.feeder.Feeder`` (substation phases 0, 1, 2 are the slack)."""
        return cls(ctx, fd.n_bus, fd.seg_from, fd.seg_to, fd.z_seg, [0, 1, 2], fd.v_slack, fd.wye_nodes,
                   fd.delta_nodes, **setup)

    def close(self) -> None:
        if self.h:
            L.lib().pf_dist_network_destroy(self.h)
            self.h = c_void_p()

    def solve(self, s_wye: torch.Tensor, s_delta: torch.Tensor, *, stream=None, **opts) -> DistResult:
        """Batched Z-bus fixed point from v0; see pf_dist_solve."""
        n = self.n_node
        ld = _ld((s_wye, n, torch.complex128, "s_wye"), (s_delta, n, torch.complex128, "s_delta"))
        B = int(s_wye.shape[0])
        dev = s_wye.device
        v = torch.empty_strided((B, n), (ld, 1), dtype=torch.complex128, device=dev)
        res = DistResult(v=v, iters=torch.empty(B, dtype=torch.int32, device=dev),
                         converged=torch.empty(B, dtype=torch.uint8, device=dev),
                         mismatch=torch.empty(B, dtype=torch.float64, device=dev),
                         sum_abs_change=torch.empty(B, dtype=torch.float64, device=dev))
        o = L.opts(**opts)
        L.call("pf_dist_solve", self.h, byref(o), B, ld, _dptr(s_wye), _dptr(s_delta), _dptr(res.v),
               _dptr(res.iters), _dptr(res.converged), _dptr(res.mismatch), _dptr(res.sum_abs_change),
               _stream(stream))
        return res


@dataclass
class EngineResult:
    v: np.ndarray            # complex128 (n, row)
    iters: np.ndarray        # int32 (n,)
    converged: np.ndarray    # uint8 (n,)
    mismatch: np.ndarray     # float64 (n,)
    times: np.ndarray        # float64 (3,): submitted, admitted, harvested (s since engine creation)


class Engine:
    """Step-level continuous-batching serving engine over one network; see
    pf_engine_create.

    ``n_streams`` >= 1: request-driven (``submit`` / ``poll`` / ``fetch``);
    ``n_streams`` = 0: caller-driven (``admit`` / ``step`` / ``harvest``).
    Host numpy arrays in and out: scenarios arrive from the host, and the
    engine stages them through its own pinned buffers into device slots.
    """

    def __init__(self, network, hbm_bytes: int, n_streams: int = 2, **opts):
        self.network = network
        self.kind = "tx" if isinstance(network, TxNetwork) else "dist"
        self.row = network.n_bus if self.kind == "tx" else network.n_node
        tx, dist = (network.h, None) if self.kind == "tx" else (None, network.h)
        self._o = L.opts(**opts)
        sb = ctypes.c_uint64()
        L.call("pf_engine_slot_bytes", tx, dist, byref(self._o), byref(sb))
        self.slot_bytes = int(sb.value)
        h = c_void_p()
        L.call("pf_engine_create", network.ctx.h, tx, dist, int(hbm_bytes), int(n_streams), byref(self._o), byref(h))
        self.h = h
        self._held: dict[int, list] = {}   # submitted requests' input arrays, until fetched

    def _inputs(self, inputs) -> tuple[int, list, list]:
        want = 3 if self.kind == "tx" else 2
        if len(inputs) != want:
            raise ValueError(f"expected {want} input arrays")
        dt = np.float64 if self.kind == "tx" else np.complex128
        arrs = [np.ascontiguousarray(a, dtype=dt) for a in inputs]
        n = int(arrs[0].shape[0])
        for a in arrs:
            if a.shape != (n, self.row):
                raise ValueError(f"inputs must have shape ({n}, {self.row})")
        return n, arrs, [_hptr(a) for a in arrs] + [None] * (3 - want)

    def submit(self, rid: int, *inputs: np.ndarray) -> None:
        """Queue request ``rid``: (p, q, vm) float64 (n, n_bus) or (s_wye, s_delta) complex128 (n, n_node).

        The engine reads the inputs when it admits the request; the arrays
        (or their contiguous copies) are held here until the request is
        fetched.  The caller must not change them before that."""
        n, arrs, ptrs = self._inputs(inputs)
        L.call("pf_engine_submit", self.h, int(rid), n, *ptrs)
        self._held[int(rid)] = arrs

    def admit(self, slots, *inputs: np.ndarray, stream=None) -> None:
        """Caller-driven: place scenarios (inputs as for ``submit``) into free ``slots``."""
        n, _arrs, ptrs = self._inputs(inputs)
        sl = np.ascontiguousarray(slots, dtype=np.int32)
        if sl.shape != (n,):
            raise ValueError("one slot per scenario")
        L.call("pf_engine_admit", self.h, n, _hptr(sl), *ptrs, _stream(stream))

    def step(self, iters: int = 1, stream=None) -> tuple[list[int], int]:
        """Caller-driven: one step; returns (slots that finished, scenarios still iterating)."""
        ms = self.info()["max_slots"]
        done = np.zeros(ms, dtype=np.int32)
        nd, na = c_int32(), c_int32()
        L.call("pf_engine_step", self.h, int(iters), ms, _hptr(done), byref(nd), byref(na), _stream(stream))
        return [int(x) for x in done[: nd.value]], na.value

    def harvest(self, slots, stream=None) -> EngineResult:
        """Caller-driven: results of finished ``slots`` (in that order); frees the slots."""
        sl = np.ascontiguousarray(slots, dtype=np.int32)
        n = int(sl.shape[0])
        res = EngineResult(v=np.empty((n, self.row), dtype=np.complex128), iters=np.empty(n, dtype=np.int32),
                           converged=np.empty(n, dtype=np.uint8), mismatch=np.empty(n),
                           times=np.zeros(3))
        L.call("pf_engine_harvest", self.h, n, _hptr(sl), _hptr(res.v), _hptr(res.iters), _hptr(res.converged),
               _hptr(res.mismatch), _stream(stream))
        return res

    def poll(self, max_ids: int = 256, timeout: float = 0.0) -> list[int]:
        ids = np.zeros(max(1, max_ids), dtype=np.int64)
        cnt = c_int32()
        L.call("pf_engine_poll", self.h, int(max_ids), _hptr(ids), float(timeout), byref(cnt))
        return [int(i) for i in ids[: cnt.value]]

    def fetch(self, rid: int) -> EngineResult:
        n = c_int32()
        L.call("pf_engine_request_size", self.h, int(rid), byref(n))
        n = n.value
        res = EngineResult(v=np.empty((n, self.row), dtype=np.complex128), iters=np.empty(n, dtype=np.int32),
                           converged=np.empty(n, dtype=np.uint8), mismatch=np.empty(n),
                           times=np.empty(3))
        try:
            L.call("pf_engine_fetch", self.h, int(rid), _hptr(res.v), _hptr(res.iters), _hptr(res.converged),
                   _hptr(res.mismatch), _hptr(res.times))
        except L.PfError as e:
            if e.status == L.PF_HIP_ERROR:   # the engine forgot the failed request
                self._held.pop(int(rid), None)
            raise
        self._held.pop(int(rid), None)
        return res

    def info(self) -> dict:
        ms, q, fl = c_int32(), c_int32(), c_int32()
        sb, jobs, sc = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        L.call("pf_engine_info", self.h, byref(ms), byref(sb), byref(q), byref(fl), byref(jobs), byref(sc))
        return {"max_slots": ms.value, "slot_bytes": sb.value, "queued": q.value, "occupied": fl.value,
                "steps": jobs.value, "scenarios": sc.value}

    def close(self) -> None:
        if self.h:
            L.lib().pf_engine_destroy(self.h)
            self.h = c_void_p()
        self._held = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def precision(name: str) -> int:
    return {"fp64": L.PF_FP64, "mixed": L.PF_MIXED}[name]
