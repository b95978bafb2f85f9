"""pf_tx_solve_noalloc (workspace in the library's fixed device array) against
pf_tx_solve (network-owned workspace) through the C ABI: the same kernels, so
every output must agree bit for bit, on consecutive calls that reuse the
array with a smaller input each time (its stale contents from the larger
call must not leak into the next)."""
import numpy as np
import pytest

from tests.gpu_common import say, to_dev
from workloads import transmission as tx

pytestmark = pytest.mark.gpu


def _inputs(grid, cfg, batch, seed):
    b = tx.make_batch(grid, cfg, batch=batch, seed=seed)
    return to_dev(b.p_inj), to_dev(b.q_inj), to_dev(b.vm_set)


def _same(a, b, label):
    for field in ("v", "newton_iters", "gmres_iters", "converged", "mismatch", "work_bytes"):
        x = getattr(a, field).cpu().numpy()
        y = getattr(b, field).cpu().numpy()
        assert x.shape == y.shape, (label, field)
        assert np.array_equal(x, y), f"{label}: {field} differs"


def test_noalloc_matches_solve_on_consecutive_calls():
    import torch
    from paper_2605_14103_amd import _lib as L
    from paper_2605_14103_amd import pf

    assert torch.cuda.is_available()
    ctx = pf.Context(0)
    cases = [(tx.TX2000, 40, "fp64"), (tx.TX2000, 9, "mixed"), (tx.TX30, 7, "fp64")]
    nets = {}
    try:
        for cfg, batch, prec in cases:
            say(f"noalloc {cfg.name} batch {batch} {prec}")
            if cfg.name not in nets:
                grid = tx.make_grid(cfg)
                nets[cfg.name] = (grid, pf.TxNetwork.from_grid(ctx, grid))
            grid, net = nets[cfg.name]
            p, q, vm = _inputs(grid, cfg, batch, seed=7 + batch)
            out = net._out(None, batch, grid.n_bus, p.device)
            net.solve_noalloc(p, q, vm, out=out, precision=pf.precision(prec))
            ref = net.solve(p, q, vm, precision=pf.precision(prec))
            torch.cuda.synchronize()
            _same(out, ref, f"{cfg.name} batch {batch} {prec}")
            assert out.converged.cpu().numpy().all()
            assert out.mismatch.cpu().numpy().max() <= 1e-8
        # a batch beyond the array is refused on the host, before any launch
        grid, net = nets["tx2000"]
        p, q, vm = _inputs(grid, tx.TX2000, 64, seed=1)
        with pytest.raises(L.PfError) as ei:
            net.solve_noalloc(p, q, vm, out=net._out(None, 64, grid.n_bus, p.device))
        assert ei.value.status == L.PF_INVALID_ARG
        with pytest.raises(L.PfError) as ei:
            net.solve_noalloc(p[:2], q[:2], vm[:2], out=net._out(None, 2, grid.n_bus, p.device), nr_direct=1)
        assert ei.value.status == L.PF_INVALID_ARG
    finally:
        for _, net in nets.values():
            net.close()
        ctx.close()
