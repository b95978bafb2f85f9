"""Host-side checks of the device library that need no GPU."""
import os
import re
import subprocess

import pytest

from paper_2605_14103_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libfile():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libpfx.so is not built (python -m paper_2605_14103_amd.build)")
    return _lib.LIB_PATH


def test_library_exports_every_declared_symbol(libfile):
    out = subprocess.run(["nm", "-D", "--defined-only", libfile], capture_output=True, text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing


def test_library_loads_and_binding_matches_header(libfile):
    h = _lib.lib()
    for name in declared_functions():
        assert hasattr(h, name)
    assert set(_lib.exported_names()) == set(declared_functions())


def test_defaults_and_option_struct():
    o = _lib.opts()
    assert o.precision == _lib.PF_FP64 and o.tol == 1e-8 and o.max_newton == 20
    assert o.gmres_restart == 30 and o.zbus_max_iter == 100 and o.precond_block == 0
    assert o.zbus_sparse == 0 and o.nr_direct == 0 and o.gmres_rtol == 0.0  # 0 selects the default 1e-3
    assert o.step_iters == 1 and o.zbus_async == 0 and o.forcing == 1 and o.forcing_max == 0.01
    with pytest.raises(TypeError):
        _lib.opts(not_an_option=1)


def test_ybus_builder_matches_definition():
    """The library's admittance builder on a 3-bus triangle, against the pi-model sums."""
    import ctypes

    import numpy as np

    f = np.array([0, 1, 0], dtype=np.int32)
    t = np.array([1, 2, 2], dtype=np.int32)
    r = np.array([0.01, 0.02, 0.03])
    x = np.array([0.1, 0.2, 0.3])
    b = np.array([0.02, 0.0, 0.04])
    cap = 9
    ptr = np.zeros(4, dtype=np.int32)
    col = np.zeros(cap, dtype=np.int32)
    yre = np.zeros(cap)
    yim = np.zeros(cap)
    nnz = ctypes.c_int32()
    P = lambda a: ctypes.c_void_p(a.ctypes.data)  # noqa: E731
    _lib.call("pf_tx_ybus_from_branches", 3, 3, P(f), P(t), P(r), P(x), P(b), cap, P(ptr), P(col), P(yre),
              P(yim), ctypes.byref(nnz))
    Y = np.zeros((3, 3), dtype=complex)
    for i in range(3):
        for p in range(ptr[i], ptr[i + 1]):
            Y[i, col[p]] = yre[p] + 1j * yim[p]
    ys = 1 / (r + 1j * x)
    E = np.zeros((3, 3), dtype=complex)
    for k in range(3):
        E[f[k], f[k]] += ys[k] + 0.5j * b[k]
        E[t[k], t[k]] += ys[k] + 0.5j * b[k]
        E[f[k], t[k]] -= ys[k]
        E[t[k], f[k]] -= ys[k]
    assert nnz.value == 9
    np.testing.assert_allclose(Y, E, rtol=1e-15, atol=1e-15)
    # too small a capacity is an error that still reports the needed size
    small = ctypes.c_int32()
    st = _lib.lib().pf_tx_ybus_from_branches(3, 3, P(f), P(t), P(r), P(x), P(b), 2, P(ptr), P(col), P(yre),
                                              P(yim), ctypes.byref(small))
    assert st == _lib.PF_INVALID_ARG and small.value == 9
    bad = f.copy()
    bad[0] = 7
    st = _lib.lib().pf_tx_ybus_from_branches(3, 3, P(bad), P(t), P(r), P(x), P(b), cap, P(ptr), P(col),
                                              P(yre), P(yim), ctypes.byref(small))
    assert st == _lib.PF_INVALID_ARG and b"out of range" in _lib.lib().pf_last_error()


def test_feeder_ybus_builder_matches_oracle_definition():
    """The library's three-phase builder against a dense assembly of inv(z) blocks."""
    import ctypes

    import numpy as np

    from workloads import feeder as fdm
    cfg = fdm.FeederConfig("feeder12", n_bus=12, max_depth=25, batch=1, seed=5)
    fd = fdm.make_feeder(cfg)
    n = fd.n_node
    cap = 3 * n + 18 * fd.n_seg
    ptr = np.zeros(n + 1, dtype=np.int32)
    col = np.zeros(cap, dtype=np.int32)
    yre = np.zeros(cap)
    yim = np.zeros(cap)
    nnz = ctypes.c_int32()
    z = np.ascontiguousarray(fd.z_seg)
    P = lambda a: ctypes.c_void_p(a.ctypes.data)  # noqa: E731
    _lib.call("pf_dist_ybus_from_segments", fd.n_bus, fd.n_seg, P(fd.seg_from), P(fd.seg_to), P(z), cap,
              P(ptr), P(col), P(yre), P(yim), ctypes.byref(nnz))
    Y = np.zeros((n, n), dtype=complex)
    for i in range(n):
        for p in range(ptr[i], ptr[i + 1]):
            Y[i, col[p]] = yre[p] + 1j * yim[p]
    E = np.zeros((n, n), dtype=complex)
    for s in range(fd.n_seg):
        y = np.linalg.inv(fd.z_seg[s])
        a, c = 3 * fd.seg_from[s], 3 * fd.seg_to[s]
        E[a:a + 3, a:a + 3] += y
        E[c:c + 3, c:c + 3] += y
        E[a:a + 3, c:c + 3] -= y
        E[c:c + 3, a:a + 3] -= y
    assert np.max(np.abs(Y - E)) <= 1e-12 * np.max(np.abs(E))


def _lib_ybus(grid):
    """The library's CSR of a grid's admittance matrix (host arrays)."""
    import ctypes

    import numpy as np

    P = lambda a: ctypes.c_void_p(a.ctypes.data)  # noqa: E731
    n, nb = grid.n_bus, int(grid.f.shape[0])
    cap = n + 2 * nb
    ptr = np.zeros(n + 1, dtype=np.int32)
    col = np.zeros(cap, dtype=np.int32)
    yre = np.zeros(cap)
    yim = np.zeros(cap)
    nnz = ctypes.c_int32()
    f, t = grid.f.astype(np.int32), grid.t.astype(np.int32)
    _lib.call("pf_tx_ybus_from_branches", n, nb, P(f), P(t), P(grid.r), P(grid.x), P(grid.b), cap, P(ptr),
              P(col), P(yre), P(yim), ctypes.byref(nnz))
    k = nnz.value
    return ptr, col[:k].copy(), yre[:k].copy(), yim[:k].copy()


def _switch(grid, csr, on, ldy=None):
    import ctypes

    import numpy as np

    P = lambda a: ctypes.c_void_p(a.ctypes.data)  # noqa: E731
    ptr, col, yre, yim = csr
    nnz = int(col.shape[0])
    ldy = nnz if ldy is None else ldy
    out = np.full((on.shape[0], ldy), np.nan, dtype=np.complex128)
    f, t = grid.f.astype(np.int32), grid.t.astype(np.int32)
    on = np.ascontiguousarray(on, dtype=np.uint8)
    st = _lib.lib().pf_tx_ybus_switch(grid.n_bus, nnz, P(ptr), P(col), P(yre), P(yim), int(f.shape[0]), P(f),
                                      P(t), P(grid.r), P(grid.x), P(grid.b), int(on.shape[0]), P(on), ldy,
                                      P(out))
    return st, out


def test_ybus_switch_matches_oracle_admittance():
    """Branch switching on the 30-bus grid: each scenario's values, read back as
    a dense matrix, equal the oracle's admittance matrix built from the branches
    left in service (two outages per scenario, plus the all-in-service case)."""
    import numpy as np

    from oracle import nr as onr
    from workloads import transmission as tx

    grid = tx.make_grid(tx.TX30)
    csr = _lib_ybus(grid)
    ptr, col = csr[0], csr[1]
    on = tx.make_outages(grid, 12, n_out=2, seed=5)
    on[0] = 1
    st, vals = _switch(grid, csr, on, ldy=int(col.shape[0]) + 3)
    assert st == _lib.PF_OK
    assert np.isnan(vals[:, -3:]).all()  # padding of each row untouched
    for s in range(on.shape[0]):
        Y = np.zeros((grid.n_bus, grid.n_bus), dtype=complex)
        for i in range(grid.n_bus):
            for p in range(ptr[i], ptr[i + 1]):
                Y[i, col[p]] += vals[s, p]
        m = on[s].astype(bool)
        ref = onr.ybus(grid.n_bus, grid.f[m], grid.t[m], grid.r[m], grid.x[m], grid.b[m]).toarray()
        np.testing.assert_allclose(Y, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    # all in service: the base values exactly
    np.testing.assert_array_equal(vals[0, :col.shape[0]], csr[2] + 1j * csr[3])


def test_ybus_switch_errors():
    import ctypes

    import numpy as np

    from workloads import transmission as tx

    grid = tx.make_grid(tx.TX30)
    csr = _lib_ybus(grid)
    on = np.ones((2, grid.f.shape[0]), dtype=np.uint8)
    st, _ = _switch(grid, csr, on, ldy=int(csr[1].shape[0]) - 1)
    assert st == _lib.PF_INVALID_ARG and b"ldy" in _lib.lib().pf_last_error()
    # a branch whose entries are not in the pattern
    import dataclasses
    f = grid.f.copy()
    t = grid.t.copy()
    pairs = set(zip(f.tolist(), t.tolist())) | set(zip(t.tolist(), f.tolist()))
    a, c = next((i, j) for i in range(grid.n_bus) for j in range(grid.n_bus) if i != j and (i, j) not in pairs)
    f[0], t[0] = a, c
    g2 = dataclasses.replace(grid, f=f, t=t)
    st, _ = _switch(g2, csr, on)
    assert st == _lib.PF_INVALID_ARG and b"pattern" in _lib.lib().pf_last_error()
    # zero scenarios is a no-op
    st, out = _switch(grid, csr, on[:0])
    assert st == _lib.PF_OK and out.shape[0] == 0
    del ctypes
