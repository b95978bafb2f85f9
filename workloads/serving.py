"""Seeded request trace for the serving mix.

Requests arrive as a Poisson process (rate ``lam`` per second) and each picks
one of the registered networks uniformly and carries a log-uniform number of
scenarios in [1, 512].  Each request's scenarios are drawn with that network's
own batch generator, seeded per request, so a request can be regenerated alone.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Request:
    rid: int
    t_arrive: float            # seconds from trace start
    network: int               # index into the trace's network list
    n_scen: int
    seed: int


@dataclass(frozen=True)
class ServingConfig:
    name: str = "serving_mix"
    lam: float = 2000.0
    n_requests: int = 20000
    max_scen: int = 512
    n_networks: int = 3
    seed: int = 4


SERVING = ServingConfig()


def make_trace(cfg: ServingConfig = SERVING, n_requests: int | None = None,
               lam: float | None = None) -> list[Request]:
    rng = np.random.default_rng(cfg.seed)
    n = cfg.n_requests if n_requests is None else int(n_requests)
    rate = cfg.lam if lam is None else float(lam)
    gaps = rng.exponential(1.0 / rate, n)
    t = np.cumsum(gaps) - gaps[0]
    net = rng.integers(0, cfg.n_networks, n)
    k = np.floor(np.exp(rng.uniform(0.0, np.log(cfg.max_scen + 1), n))).astype(np.int64)
    k = np.clip(k, 1, cfg.max_scen)
    seeds = rng.integers(1, 2**31 - 1, n)
    return [Request(rid=i, t_arrive=float(t[i]), network=int(net[i]), n_scen=int(k[i]),
                    seed=int(seeds[i])) for i in range(n)]
