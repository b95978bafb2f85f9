"""pfx: batched AC power flow on AMD MI355X (gfx950).

Device library (HIP kernels behind a C ABI, include/pfx.h) with a thin Python
binding.  Importing the package does not load the library; the first call does,
and it fails loudly if the library has not been built
(``python -m paper_2605_14103_amd.build``).
"""
from ._lib import PF_FP64, PF_MIXED, PfError  # noqa: F401

__all__ = ["PF_FP64", "PF_MIXED", "PfError"]
