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
