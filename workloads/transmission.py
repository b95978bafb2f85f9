"""Seeded synthetic meshed transmission grids and their scenario batches.

This module only draws random numbers and lays them out.  It holds none of the
power-flow arithmetic (no admittance matrix, no mismatch, no solve); the GPU
library and the CPU oracle each build what they need from these raw arrays.

The workloads stand in for the paper's transmission test cases (Sec. III), which
are not available here: a meshed grid (a spanning tree anchored on the generator
buses plus extra lines), pi-model lines, PQ loads with a fixed power factor and
PV generators with voltage set-points.  Scenario batches perturb the loads (and PV dispatch) per scenario,
as the paper's case studies do with random load multipliers (Sec. III).

Array layout: every per-scenario, per-bus quantity is ``[batch, n_bus]``
(scenario-major, one contiguous row per scenario), the layout the device
library consumes.
Injections follow the generator convention (generation minus load).
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass, field

import numpy as np

PQ, PV, SLACK = 0, 1, 2


@dataclass
class TxGrid:
    """A transmission network as raw branch and bus data (per unit)."""

    n_bus: int
    bus_type: np.ndarray      # int8 [n]: 0 = PQ, 1 = PV, 2 = slack (exactly one)
    f: np.ndarray             # int32 [n_branch] from-bus
    t: np.ndarray             # int32 [n_branch] to-bus
    r: np.ndarray             # float64 series resistance
    x: np.ndarray             # float64 series reactance
    b: np.ndarray             # float64 total line charging (split half per end)
    vm_set: np.ndarray        # float64 [n]: PV / slack set-point, 1.0 at PQ buses
    p_load: np.ndarray        # float64 [n]: base active load (PQ buses only)
    q_load: np.ndarray        # float64 [n]: base reactive load (PQ buses only)
    p_gen: np.ndarray         # float64 [n]: base PV dispatch (PV buses only)
    slack: int
    name: str = ""

    @property
    def n_branch(self) -> int:
        return int(self.f.shape[0])

    @property
    def n_pv(self) -> int:
        return int(np.sum(self.bus_type == PV))

    @property
    def n_pq(self) -> int:
        return int(np.sum(self.bus_type == PQ))


@dataclass
class TxBatch:
    """A batch of scenarios on one grid, one row per scenario."""

    p_inj: np.ndarray         # float64 [B, n]: scheduled active injection
    q_inj: np.ndarray         # float64 [B, n]: scheduled reactive injection
    vm_set: np.ndarray        # float64 [B, n]: |V| set-points (PV, slack); 1.0 elsewhere
    meta: dict = field(default_factory=dict)

    @property
    def batch(self) -> int:
        return int(self.p_inj.shape[0])


@dataclass(frozen=True)
class TxConfig:
    """Recipe for one synthetic grid and its scenario batch."""

    name: str
    n_bus: int
    n_pv: int
    n_branch: int
    batch: int
    seed: int
    perturbation: str          # "lognormal" (one factor per scenario) or "uniform" (per bus)
    sigma: float = 0.1         # lognormal sigma
    spread: float = 0.2        # half-width of the uniform multiplier
    # Each PV unit is dispatched to the load it serves times (1 + allowance), so
    # that the slack bus is not left to carry all network losses alone.  The
    # value was picked by running the oracle's base case; the workload tests
    # check that every scenario then converges.
    loss_allowance: float = 0.02


# 30 buses (1 slack, 5 PV, 24 PQ), 41 branches, 64 scenarios scaled by one
# lognormal(0, 0.1) factor each.
TX30 = TxConfig("tx30", n_bus=30, n_pv=5, n_branch=41, batch=64, seed=30,
                perturbation="lognormal", sigma=0.1)
# 2000 buses (1 slack, 300 PV, 1699 PQ), average nodal degree 2.6 -> 2600
# branches, 1024 scenarios with an independent +/-20% multiplier per bus.
TX2000 = TxConfig("tx2000", n_bus=2000, n_pv=300, n_branch=2600, batch=1024, seed=2000,
                  perturbation="uniform", spread=0.2)
# The adjoint workload: the 2000-bus grid with 256 scenarios.
TX2000_ADJ = TxConfig("tx2000_adj", n_bus=2000, n_pv=300, n_branch=2600, batch=256, seed=2000,
                      perturbation="uniform", spread=0.2)


def anchored_mesh(n_source: int, n: int, n_branch: int, rng: np.random.Generator):
    """Source-anchored meshed topology over buses 0..n-1 (sources are 0..n_source-1).

    * backbone: a random recursive tree over the source buses;
    * every other bus gets one line to a uniformly drawn source bus;
    * extra lines first pair up degree-one buses at random (so no bus hangs
      off the grid by a single line), then join uniform random pairs.
    No self-loops, no parallel lines.  Returns (f, t) int64 arrays.
    """
    if n_branch < n - 1:
        raise ValueError("need at least n-1 branches for a connected grid")
    if n_branch > n * (n - 1) // 2:
        raise ValueError("too many branches for a simple graph")
    edges = []
    seen = set()
    deg = np.zeros(n, dtype=np.int64)

    def add(a, c):
        key = (min(a, c), max(a, c))
        if a == c or key in seen:
            return
        seen.add(key)
        edges.append((a, c))
        deg[a] += 1
        deg[c] += 1

    for k in range(1, n_source):
        add(int(rng.integers(0, k)), k)
    for k in range(n_source, n):
        add(int(rng.integers(0, n_source)), k)
    leaves = rng.permutation(np.flatnonzero(deg == 1))
    for i in range(0, leaves.shape[0] - 1, 2):
        if len(edges) >= n_branch:
            break
        add(int(leaves[i]), int(leaves[i + 1]))
    while len(edges) < n_branch:
        a, c = (int(v) for v in rng.integers(0, n, size=2))
        add(a, c)
    e = np.asarray(edges, dtype=np.int64)
    return e[:, 0].copy(), e[:, 1].copy()


def _adjacency(n, f, t):
    adj = [[] for _ in range(n)]
    for a, c in zip(f.tolist(), t.tolist()):
        adj[a].append(c)
        adj[c].append(a)
    return adj


def _nearest_source(adj, sources):
    """Owning source of every bus: the first source a breadth-first search reaches it from."""
    owner = np.full(len(adj), -1, dtype=np.int64)
    queue = deque()
    for s in sources:
        owner[s] = s
        queue.append(s)
    while queue:
        u = queue.popleft()
        for w in adj[u]:
            if owner[w] < 0:
                owner[w] = owner[u]
                queue.append(w)
    return owner


def make_grid(cfg: TxConfig) -> TxGrid:
    """Draw one grid from its config (deterministic in ``cfg.seed``).

    Topology: ``anchored_mesh`` with the slack and PV buses as sources, then a
    seeded relabelling of all buses.  Slack: the highest-degree source (lowest
    label on ties); the other sources are PV buses.  Loads on PQ buses only.
    Dispatch: every PQ bus is served by its nearest source in hops; each PV
    unit is dispatched to its served load times (1 + loss allowance), and the
    slack covers its own served load and the remaining losses.
    """
    rng = np.random.default_rng(cfg.seed)
    n = cfg.n_bus
    n_src = cfg.n_pv + 1
    f0, t0 = anchored_mesh(n_src, n, cfg.n_branch, rng)
    label = rng.permutation(n)
    f = label[f0].astype(np.int32)
    t = label[t0].astype(np.int32)
    nbr = f.shape[0]
    r = rng.uniform(0.01, 0.08, nbr)
    x = r * rng.uniform(2.0, 6.0, nbr)
    b = rng.uniform(0.0, 0.05, nbr)

    sources = np.sort(label[:n_src])
    deg = np.bincount(np.concatenate([f, t]), minlength=n)
    slack = int(sources[np.flatnonzero(deg[sources] == deg[sources].max())[0]])
    pv = sources[sources != slack]

    bus_type = np.zeros(n, dtype=np.int8)
    bus_type[pv] = PV
    bus_type[slack] = SLACK
    pq = np.flatnonzero(bus_type == PQ)

    vm_set = np.ones(n)
    vm_set[pv] = rng.uniform(1.0, 1.05, pv.shape[0])

    p_load = np.zeros(n)
    q_load = np.zeros(n)
    p_load[pq] = rng.uniform(0.05, 0.4, pq.shape[0])
    q_load[pq] = 0.3 * p_load[pq]

    owner = _nearest_source(_adjacency(n, f, t), [slack] + pv.tolist())
    served = np.zeros(n)
    np.add.at(served, owner, p_load)
    p_gen = np.zeros(n)
    p_gen[pv] = (1.0 + cfg.loss_allowance) * served[pv]
    return TxGrid(n_bus=n, bus_type=bus_type, f=f, t=t, r=r, x=x, b=b, vm_set=vm_set,
                  p_load=p_load, q_load=q_load, p_gen=p_gen, slack=slack, name=cfg.name)


def make_batch(grid: TxGrid, cfg: TxConfig, batch: int | None = None, seed: int | None = None) -> TxBatch:
    """Draw a scenario batch (deterministic in ``seed``, default ``cfg.seed + 1``)."""
    B = cfg.batch if batch is None else int(batch)
    rng = np.random.default_rng(cfg.seed + 1 if seed is None else seed)
    n = grid.n_bus
    if cfg.perturbation == "lognormal":
        fac = np.exp(rng.normal(0.0, cfg.sigma, B))
        load_mult = np.broadcast_to(fac[:, None], (B, n))
        gen_mult = np.ones((B, n))
    elif cfg.perturbation == "uniform":
        load_mult = rng.uniform(1.0 - cfg.spread, 1.0 + cfg.spread, (B, n))
        gen_mult = rng.uniform(1.0 - cfg.spread, 1.0 + cfg.spread, (B, n))
    else:
        raise ValueError(cfg.perturbation)
    p = grid.p_gen[None, :] * gen_mult - grid.p_load[None, :] * load_mult
    q = -grid.q_load[None, :] * load_mult
    vm = np.broadcast_to(grid.vm_set[None, :], (B, n))
    return TxBatch(p_inj=np.ascontiguousarray(p), q_inj=np.ascontiguousarray(q),
                   vm_set=np.ascontiguousarray(vm), meta={"config": cfg.name, "batch": B})


def two_bus(r: float, x: float, p_load: float, q_load: float, batch: int = 1) -> tuple[TxGrid, TxBatch]:
    """The 2-bus case: slack at bus 0, one PQ load at bus 1, one line without charging."""
    grid = TxGrid(n_bus=2, bus_type=np.array([SLACK, PQ], dtype=np.int8),
                  f=np.array([0], dtype=np.int32), t=np.array([1], dtype=np.int32),
                  r=np.array([r]), x=np.array([x]), b=np.array([0.0]),
                  vm_set=np.ones(2), p_load=np.array([0.0, p_load]),
                  q_load=np.array([0.0, q_load]), p_gen=np.zeros(2), slack=0, name="two_bus")
    p = np.zeros((batch, 2))
    q = np.zeros((batch, 2))
    p[:, 1] = -p_load
    q[:, 1] = -q_load
    return grid, TxBatch(p_inj=p, q_inj=q, vm_set=np.ones((batch, 2)))


def zero_load(grid: TxGrid, batch: int = 1) -> TxBatch:
    """No load and no dispatch anywhere, all set-points 1.0."""
    n = grid.n_bus
    return TxBatch(p_inj=np.zeros((batch, n)), q_inj=np.zeros((batch, n)),
                   vm_set=np.ones((batch, n)))


def make_outages(grid: TxGrid, batch: int, n_out: int = 1, seed: int = 0) -> np.ndarray:
    """Branch status per scenario for topology-action batches: ``branch_on``
    uint8 [batch, n_branch], 1 = in service.  Each scenario takes ``n_out``
    distinct branches out of service, drawn uniformly among those whose removal
    keeps every bus connected to the slack (redrawn otherwise), so each
    scenario stays a well-posed power flow.  Pure data generation (a graph
    connectivity test, no electrical quantity)."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    rng = np.random.default_rng(seed)
    n, nb = grid.n_bus, int(grid.f.shape[0])
    on = np.ones((batch, nb), dtype=np.uint8)

    def connected(mask):
        g = coo_matrix((np.ones(int(mask.sum())), (grid.f[mask], grid.t[mask])), shape=(n, n))
        return connected_components(g, directed=False)[0] == 1

    for s in range(batch):
        mask = np.ones(nb, dtype=bool)
        taken = 0
        for _ in range(100 * max(n_out, 1)):
            if taken == n_out:
                break
            k = int(rng.integers(0, nb))
            if not mask[k]:
                continue
            mask[k] = False
            if connected(mask):
                taken += 1
            else:
                mask[k] = True
        if taken != n_out:
            raise ValueError(f"could not take {n_out} branches out without islanding a bus")
        on[s] = mask
    return on
