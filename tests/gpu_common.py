"""Helpers shared by the GPU tests (imported only by tests marked gpu)."""
import sys

import numpy as np


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def angle_err(v_gpu, v_ref):
    """Max |angle difference| (rad) and max ||V| difference| (pu), elementwise."""
    d_ang = np.abs(np.angle(v_gpu * np.conj(v_ref)))
    d_mag = np.abs(np.abs(v_gpu) - np.abs(v_ref))
    return float(d_ang.max()), float(d_mag.max())


def spread_cols(batch: int, k: int = 32) -> np.ndarray:
    """k scenario indices spread evenly over a batch, first and last included."""
    return np.unique(np.linspace(0, batch - 1, min(k, batch)).round().astype(np.int64))


# Power flow has several solutions; the one both sides must reach from a flat
# start (transmission) or from the no-load voltage (feeder) is the high-voltage
# one.  Every scenario of a full-batch GPU run is held to these floors, not just
# the ones compared with the oracle.
HV_FLOOR_TX = 0.7      # pu, transmission bus voltages
HV_FLOOR_FEEDER = 0.85  # pu, feeder phase voltages


def assert_high_voltage(v_gpu: np.ndarray, floor: float, label: str) -> None:
    vmin = np.abs(v_gpu).min(axis=1)
    worst = int(np.argmin(vmin))
    say(f"{label}: min |V| over all {v_gpu.shape[0]} scenarios {vmin[worst]:.4f} pu (scenario {worst})")
    assert np.isfinite(vmin).all() and vmin.min() > floor, f"{label}: scenario {worst} at {vmin[worst]:.4f} pu"
