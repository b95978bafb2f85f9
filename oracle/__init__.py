"""Plain, slow, obviously correct FP64 CPU oracle for batched AC power flow.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and the
benchmark's CPU-baseline leg may import anything here.  The GPU library never
calls into this package and this package never calls into the GPU library;
the two share nothing but the seeded input generators in ``workloads``.

Contents
--------
nr       Newton-Raphson on a meshed grid with a sparse LU Newton step
         (Sec. II-A, eqs. (1)-(3); Jacobian blocks of eq. (4)).
zbus     The three-phase Z-bus fixed point of eq. (10) on a radial feeder,
         run literally, with wye and delta constant-power loads (Sec. II-B).
adjoint  Branch-current loss, its gradient, and the dense adjoint of the
         converged Newton-Raphson solution with respect to the injections.

Parity pins for every function live in ``tests/test_oracle_*.py``.  Nothing
here is "parity unpinned".
"""
