"""ctypes declarations for libpfx.so (the C ABI in include/pfx.h).

Loading fails loudly when the library has not been built: there is no CPU
fallback anywhere in this package.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int8, c_int32, c_int64, c_uint8, c_uint64, c_void_p

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpfx.so")

PF_OK, PF_INVALID_ARG, PF_OUT_OF_MEMORY, PF_HIP_ERROR, PF_SINGULAR_SETUP, PF_NOT_ADMITTED, PF_BAD_HANDLE = range(7)
PF_FP64, PF_MIXED = 0, 1
STATUS_NAMES = {0: "PF_OK", 1: "PF_INVALID_ARG", 2: "PF_OUT_OF_MEMORY", 3: "PF_HIP_ERROR",
                4: "PF_SINGULAR_SETUP", 5: "PF_NOT_ADMITTED", 6: "PF_BAD_HANDLE"}


class PfOpts(ctypes.Structure):
    _fields_ = [
        ("precision", c_int32),
        ("tol", c_double),
        ("max_newton", c_int32),
        ("gmres_restart", c_int32),
        ("gmres_max_restarts", c_int32),
        ("gmres_rtol", c_double),
        ("diverge", c_double),
        ("zbus_max_iter", c_int32),
        ("eps", c_double),
        ("precond_block", c_int32),
        ("factor_max_levels", c_int32),
        ("factor_max_core", c_int32),
        ("zbus_sparse", c_int32),
        ("zbus_async", c_int32),
        ("nr_direct", c_int32),
        ("step_iters", c_int32),
        ("forcing", c_int32),
        ("forcing_max", c_double),
    ]


class PfError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


P = c_void_p
I32P = POINTER(c_int32)
F64P = POINTER(c_double)

# (name, restype, argtypes); pointers to device memory are passed as c_void_p.
_SIGS = [
    ("pf_opts_default", None, [POINTER(PfOpts)]),
    ("pf_last_error", c_char_p, []),
    ("pf_context_create", c_int32, [c_int32, c_uint64, POINTER(P)]),
    ("pf_context_destroy", None, [P]),
    ("pf_context_bytes", c_uint64, [P]),
    ("pf_tx_ybus_from_branches", c_int32,
     [c_int32, c_int32, P, P, P, P, P, c_int32, P, P, P, P, I32P]),
    ("pf_tx_network_create", c_int32,
     [P, c_int32, c_int32, P, P, P, P, P, c_int32, P, P, P, P, P, POINTER(PfOpts), POINTER(P)]),
    ("pf_tx_network_destroy", None, [P]),
    ("pf_tx_network_info", c_int32, [P, I32P, I32P, I32P, I32P, I32P, I32P, I32P]),
    ("pf_tx_solve", c_int32,
     [P, POINTER(PfOpts), c_int32, c_int64, P, P, P, P, P, P, P, P, P, P]),
    ("pf_tx_solve_noalloc", c_int32,
     [P, POINTER(PfOpts), c_int32, c_int64, P, P, P, P, P, P, P, P, P, P]),
    ("pf_tx_solve_yvals", c_int32,
     [P, POINTER(PfOpts), c_int32, c_int64, P, P, P, c_int64, P, P, P, P, P, P, P, P]),
    ("pf_tx_ybus_switch", c_int32,
     [c_int32, c_int32, P, P, P, P, c_int32, P, P, P, P, P, c_int32, P, c_int64, P]),
    ("pf_tx_branch_loss", c_int32, [P, c_int32, c_int64, P, P, P, P]),
    ("pf_tx_adjoint", c_int32, [P, POINTER(PfOpts), c_int32, c_int64, P, P, P, P, P, P, P]),
    ("pf_dist_ybus_from_segments", c_int32,
     [c_int32, c_int32, P, P, P, c_int32, P, P, P, P, I32P]),
    ("pf_dist_network_create", c_int32,
     [P, c_int32, c_int32, P, P, P, P, P, P, c_int32, P, c_int32, P, POINTER(PfOpts), POINTER(P)]),
    ("pf_dist_network_destroy", None, [P]),
    ("pf_dist_network_info", c_int32, [P, I32P, I32P, I32P, I32P]),
    ("pf_dist_solve", c_int32,
     [P, POINTER(PfOpts), c_int32, c_int64, P, P, P, P, P, P, P, P]),
    ("pf_engine_slot_bytes", c_int32, [P, P, POINTER(PfOpts), POINTER(c_uint64)]),
    ("pf_engine_create", c_int32, [P, P, P, c_uint64, c_int32, POINTER(PfOpts), POINTER(P)]),
    ("pf_engine_destroy", None, [P]),
    ("pf_engine_submit", c_int32, [P, c_int64, c_int32, P, P, P]),
    ("pf_engine_poll", c_int32, [P, c_int32, P, c_double, I32P]),
    ("pf_engine_request_size", c_int32, [P, c_int64, I32P]),
    ("pf_engine_fetch", c_int32, [P, c_int64, P, P, P, P, P]),
    ("pf_engine_info", c_int32, [P, I32P, POINTER(c_uint64), I32P, I32P, POINTER(c_uint64), POINTER(c_uint64)]),
    ("pf_engine_admit", c_int32, [P, c_int32, P, P, P, P, P]),
    ("pf_engine_step", c_int32, [P, c_int32, c_int32, P, I32P, I32P, P]),
    ("pf_engine_harvest", c_int32, [P, c_int32, P, P, P, P, P, P]),
]

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2605_14103_amd.build`")
        h = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def exported_names() -> list[str]:
    return [s[0] for s in _SIGS]


def check(status: int, func: str) -> None:
    if status != PF_OK:
        msg = lib().pf_last_error()
        raise PfError(status, func, msg.decode() if msg else "")


def call(name: str, *args) -> None:
    check(getattr(lib(), name)(*args), name)


def opts(**kw) -> PfOpts:
    o = PfOpts()
    lib().pf_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o
