"""The allocation-free scaled norm (isc_scaled_norm_noalloc) against the
context's isc_scaled_norm, through the C-ABI: two calls in a row on one
device, the second on a smaller grid, each equal to the context's result
(a maximum of identically computed terms, so bit for bit); a grid above the
fixed buffer's limit is refused on the host before anything is launched."""
import numpy as np
import pytest
import torch

from paper_1811_11992_amd import inputs as I
from paper_1811_11992_amd import isc

pytestmark = pytest.mark.gpu


def _residual(name, seed):
    """F at a perturbed admissible state of workload `name` (from the HIP
    assembly), the context's norm of it, and what the free call needs."""
    wl = I.make_workload(name)
    ctx = isc.Context(wl, device="cuda:0")
    u0 = torch.tensor(wl.u0, dtype=torch.float64, device="cuda:0")
    u = torch.tensor(I.random_states(wl, seed=seed), dtype=torch.float64, device="cuda:0")
    F, _ = ctx.isc_assemble(u, u0, wl.dt)
    ref = ctx.isc_scaled_norm(F, wl.dt)
    return wl, ctx, F, ref


def test_noalloc_norm_matches_context_norm_on_two_calls():
    res = torch.full((1,), -1.0, dtype=torch.float64, device="cuda:0")
    fl = I.physics_card()
    for name, seed in (("tiny:40x30x20", 3), ("tiny:6x5x3", 4)):
        print(f"noalloc norm: {name} seed {seed}", flush=True)
        wl, ctx, F, ref = _residual(name, seed)
        st = isc.isc_scaled_norm_noalloc(wl.grid(), fl, ctx.poro, F, wl.dt, res)
        assert st == isc.ISC_OK, isc.lib().isc_last_error(None)
        torch.cuda.synchronize()
        got = float(res.item())
        assert np.isfinite(ref) and ref > 0
        assert got == ref, (name, got, ref)
        # a residual with a planted non-finite entry propagates as NaN, as in the context's norm
        F2 = F.clone()
        F2[wl.ncell // 2, 3] = float("nan")
        assert isc.isc_scaled_norm_noalloc(wl.grid(), fl, ctx.poro, F2, wl.dt, res) == isc.ISC_OK
        torch.cuda.synchronize()
        assert np.isnan(res.item()) and np.isnan(ctx.isc_scaled_norm(F2, wl.dt))
        del ctx


def test_noalloc_norm_refuses_grids_above_its_buffer():
    fl = I.physics_card()
    res = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    small = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    big = I.Grid(4096, 4097, 1, 5.0, 5.0, 2.0)       # one row more than the limit
    assert 4096 * 4097 > isc.NOALLOC_MAX_CELLS
    st = isc.isc_scaled_norm_noalloc(big, fl, small, small, 8640.0, res)
    assert st == isc.ISC_ERR_ARG
    assert b"exceed the maximum" in isc.lib().isc_last_error(None)
    assert isc.isc_scaled_norm_noalloc(I.Grid(2, 2, 2, 5.0, 5.0, 2.0), fl, small, small, 0.0, res) == isc.ISC_ERR_ARG
