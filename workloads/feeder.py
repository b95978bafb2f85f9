"""Seeded synthetic three-phase unbalanced radial feeders and their load batches.

Random draws and layout only: no admittance matrix, no impedance matrix, no
current-injection map.  The GPU library and the CPU oracle each build those.

The feeders stand in for the paper's distribution test cases (Sec. III), which
are not available here.  Every bus is three-phase; phase node ``3*bus + ph``
(ph = 0, 1, 2 for a, b, c).  Bus 0 is the substation (slack phases), the other
buses hang off a random tree of bounded depth.  Segment impedances are 3x3
complex matrices with self impedance on the diagonal and a symmetric fraction of
it off the diagonal.  Loads are constant power, either wye (phase to neutral)
or delta (phase to phase).

Per-unit system: line-to-line base 4.16 kV, three-phase base 1 MVA; per-phase
quantities use the line-to-neutral voltage base and one third of the power
base, so the impedance base is 4.16^2 / 1 = 17.3056 ohm.

Load arrays are ``[batch, n_node]`` complex (one row per scenario), in the
consumption convention.  ``s_wye[node]`` is the wye load on that phase node.
For a delta bus with nodes (a, b, c), ``s_delta[a]``, ``s_delta[b]`` and
``s_delta[c]`` hold the loads of the ab, bc and ca branches.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

V_LL_KV = 4.16
S_BASE_3PH_KVA = 1000.0
S_BASE_PH_KVA = S_BASE_3PH_KVA / 3.0
Z_BASE_OHM = V_LL_KV ** 2 / (S_BASE_3PH_KVA / 1000.0)


@dataclass
class Feeder:
    n_bus: int
    parent: np.ndarray        # int32 [n_bus]; parent[0] = -1
    depth: np.ndarray         # int32 [n_bus]
    seg_from: np.ndarray      # int32 [n_seg] parent bus
    seg_to: np.ndarray        # int32 [n_seg] child bus
    z_seg: np.ndarray         # complex128 [n_seg, 3, 3] series impedance (pu)
    load_kind: np.ndarray     # int8 [n_bus]: 0 none, 1 wye, 2 delta
    s_base_wye: np.ndarray    # complex128 [n_node] base wye loads (pu)
    s_base_delta: np.ndarray  # complex128 [n_node] base delta branch loads (pu)
    v_slack: np.ndarray       # complex128 [3] substation phase voltages (pu)
    name: str = ""

    @property
    def n_node(self) -> int:
        return 3 * self.n_bus

    @property
    def n_seg(self) -> int:
        return int(self.seg_from.shape[0])

    @property
    def wye_nodes(self) -> np.ndarray:
        buses = np.flatnonzero(self.load_kind == 1)
        return (3 * buses[:, None] + np.arange(3)[None, :]).reshape(-1).astype(np.int32)

    @property
    def delta_nodes(self) -> np.ndarray:
        buses = np.flatnonzero(self.load_kind == 2)
        return (3 * buses[:, None] + np.arange(3)[None, :]).astype(np.int32)


@dataclass
class FeederBatch:
    s_wye: np.ndarray         # complex128 [B, n_node]
    s_delta: np.ndarray       # complex128 [B, n_node]
    meta: dict = field(default_factory=dict)

    @property
    def batch(self) -> int:
        return int(self.s_wye.shape[0])


@dataclass(frozen=True)
class FeederConfig:
    name: str
    n_bus: int
    max_depth: int
    batch: int
    seed: int
    wye_share: float = 0.6
    pf: float = 0.95
    spread: float = 0.2


# 300 buses (900 phase nodes), tree depth <= 25, 4096 scenarios.
FEEDER300 = FeederConfig("feeder300", n_bus=300, max_depth=25, batch=4096, seed=300)


def _random_tree(n: int, max_depth: int, rng: np.random.Generator):
    parent = np.full(n, -1, dtype=np.int32)
    depth = np.zeros(n, dtype=np.int32)
    for k in range(1, n):
        eligible = np.flatnonzero(depth[:k] <= max_depth - 1)
        p = int(eligible[int(rng.integers(0, eligible.shape[0]))])
        parent[k] = p
        depth[k] = depth[p] + 1
    return parent, depth


def make_feeder(cfg: FeederConfig) -> Feeder:
    rng = np.random.default_rng(cfg.seed)
    n = cfg.n_bus
    parent, depth = _random_tree(n, cfg.max_depth, rng)
    seg_to = np.arange(1, n, dtype=np.int32)
    seg_from = parent[1:].astype(np.int32)
    nseg = n - 1
    r_km = rng.uniform(0.1, 0.6, nseg)
    x_km = rng.uniform(0.2, 0.8, nseg)
    length = rng.uniform(0.05, 0.5, nseg)
    kappa = rng.uniform(0.3, 0.5, (nseg, 3))          # ab, bc, ca coupling fractions
    z_self = (r_km + 1j * x_km) * length / Z_BASE_OHM
    z = np.zeros((nseg, 3, 3), dtype=np.complex128)
    for s in range(nseg):
        z[s, 0, 0] = z[s, 1, 1] = z[s, 2, 2] = z_self[s]
        z[s, 0, 1] = z[s, 1, 0] = kappa[s, 0] * z_self[s]
        z[s, 1, 2] = z[s, 2, 1] = kappa[s, 1] * z_self[s]
        z[s, 2, 0] = z[s, 0, 2] = kappa[s, 2] * z_self[s]

    load_kind = np.zeros(n, dtype=np.int8)
    loaded = rng.permutation(np.arange(1, n))
    n_wye = int(round(cfg.wye_share * (n - 1)))
    load_kind[loaded[:n_wye]] = 1
    load_kind[loaded[n_wye:]] = 2

    tan_phi = np.tan(np.arccos(cfg.pf))
    p_kw = rng.uniform(1.0, 10.0, 3 * n)
    s_node = (p_kw + 1j * p_kw * tan_phi) / S_BASE_PH_KVA
    kind_node = np.repeat(load_kind, 3)
    s_wye = np.where(kind_node == 1, s_node, 0.0).astype(np.complex128)
    s_delta = np.where(kind_node == 2, s_node, 0.0).astype(np.complex128)

    a = np.exp(-2j * np.pi / 3)
    v_slack = np.array([1.0, a, a * a], dtype=np.complex128)
    return Feeder(n_bus=n, parent=parent, depth=depth, seg_from=seg_from, seg_to=seg_to,
                  z_seg=z, load_kind=load_kind, s_base_wye=s_wye, s_base_delta=s_delta,
                  v_slack=v_slack, name=cfg.name)


def make_batch(feeder: Feeder, cfg: FeederConfig, batch: int | None = None,
               seed: int | None = None) -> FeederBatch:
    """Independent U(1 - spread, 1 + spread) multiplier per load phase and scenario."""
    B = cfg.batch if batch is None else int(batch)
    rng = np.random.default_rng(cfg.seed + 1 if seed is None else seed)
    mult = rng.uniform(1.0 - cfg.spread, 1.0 + cfg.spread, (B, feeder.n_node))
    s_wye = feeder.s_base_wye[None, :] * mult
    s_delta = feeder.s_base_delta[None, :] * mult
    return FeederBatch(s_wye=np.ascontiguousarray(s_wye), s_delta=np.ascontiguousarray(s_delta),
                       meta={"config": cfg.name, "batch": B})


def single_segment(z_self: complex, kappa: float, kind: int, s_phase: complex,
                   batch: int = 1) -> tuple[Feeder, FeederBatch]:
    """Substation plus one loaded bus on one segment with equal coupling on all pairs.

    ``kind`` 1 puts a balanced wye load ``s_phase`` on each phase, ``kind`` 2 a
    balanced delta load ``s_phase`` on each branch.
    """
    z = np.full((1, 3, 3), kappa * z_self, dtype=np.complex128)
    for p in range(3):
        z[0, p, p] = z_self
    a = np.exp(-2j * np.pi / 3)
    s = np.zeros(6, dtype=np.complex128)
    s[3:] = s_phase
    fd = Feeder(n_bus=2, parent=np.array([-1, 0], dtype=np.int32), depth=np.array([0, 1], dtype=np.int32),
                seg_from=np.array([0], dtype=np.int32), seg_to=np.array([1], dtype=np.int32), z_seg=z,
                load_kind=np.array([0, kind], dtype=np.int8),
                s_base_wye=s if kind == 1 else np.zeros(6, dtype=np.complex128),
                s_base_delta=s if kind == 2 else np.zeros(6, dtype=np.complex128),
                v_slack=np.array([1.0, a, a * a]), name="single_segment")
    sw = np.repeat(fd.s_base_wye[None, :], batch, axis=0)
    sd = np.repeat(fd.s_base_delta[None, :], batch, axis=0)
    return fd, FeederBatch(s_wye=sw, s_delta=sd)


def zero_load(feeder: Feeder, batch: int = 1) -> FeederBatch:
    z = np.zeros((batch, feeder.n_node), dtype=np.complex128)
    return FeederBatch(s_wye=z.copy(), s_delta=z.copy())
