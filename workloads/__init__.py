"""Seeded synthetic inputs shared by the device library's tests and benches and the CPU oracle.

Only random draws and array layout live here; none of the power-flow method's
arithmetic does.
"""
from . import feeder, serving, transmission  # noqa: F401
