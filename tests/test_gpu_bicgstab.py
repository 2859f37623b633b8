"""BiCGSTAB with block ILU(0) (the Krylov method of the paper's experiments)
through the C-ABI, against the oracle's BiCGSTAB and a tight oracle solve.

Tolerances: the true residual of the GPU solution, recomputed by the oracle,
<= 1.01 rtol; distance to a 1e-13 oracle GMRES solution <= 1e-5 (the systems'
conditioning, as for the GMRES solve); iteration count within a factor two
(plus five) of the oracle's BiCGSTAB, whose inner products round differently.
"""
import numpy as np
import pytest
import torch

from paper_1811_11992_amd import inputs as I
import oracle as O

pytestmark = pytest.mark.gpu

COL = np.array([1e6, 1.0, 1.0, 1.0, 100.0, 1.0, 1.0, 1000.0])   # unit size of each unknown


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _system(name, seed):
    wl = I.make_workload(name)
    m = O.Model(wl)
    u = I.random_states(wl, seed)
    F, J = m.assemble(u, wl.u0, wl.dt)
    st, Jd, Fd, _ = m.decouple(J, F)
    assert st == 0
    return wl, m, Jd, -Fd


@pytest.mark.parametrize("level", ["0", "1"])
@pytest.mark.parametrize("name,seed", [("tiny:13x7x5", 21), ("C1", 22)])
def test_bicgstab_matches_oracle(name, seed, level, monkeypatch):
    from paper_1811_11992_amd import isc
    monkeypatch.setenv("ISC_LEVEL_SWEEPS", level)
    wl, m, Jd, b = _system(name, seed)
    c = isc.Context(wl)
    x, info, st = c.isc_solve_bicgstab(_dev(Jd), _dev(b), rtol=1e-8)
    assert st == 0 and info.relres_true <= 1e-8
    xg = _host(x)
    assert np.linalg.norm(b - m.spmv(Jd, xg)) <= 1.01e-8 * np.linalg.norm(b)
    st_o, x_o, inf_o = m.bicgstab(Jd, b, rtol=1e-8)
    assert st_o == 0
    assert info.iters <= 2 * inf_o.iters + 5, (info.iters, inf_o.iters)
    st, x_ref, _ = m.gmres(Jd, b, rtol=1e-13, max_restarts=60)
    err = np.abs((xg - x_ref) / COL).max(axis=0)
    assert np.all(err <= 1e-5 * np.abs(x_ref / COL).max()), err


def test_bicgstab_exact_preconditioner_and_zero_rhs():
    """On a one-cell-wide chain BILU(0) is exact: one iteration, the dense
    solution to rounding.  A zero right-hand side returns zero at once."""
    from paper_1811_11992_amd import isc
    wl, m, Jd, b = _system("tiny:9x1x1", 41)
    c = isc.Context(wl)
    x, info, st = c.isc_solve_bicgstab(_dev(Jd), _dev(b), rtol=1e-8)
    assert st == 0 and info.iters == 1 and info.relres_true <= 1e-12
    st_o, x_o, _ = m.bicgstab(Jd, b, rtol=1e-8)
    xg = _host(x)
    assert np.abs((xg - x_o) / COL).max() <= 1e-9 * np.abs(x_o / COL).max()
    x, info, st = c.isc_solve_bicgstab(_dev(Jd), _dev(np.zeros_like(b)), rtol=1e-8)
    assert st == 0 and info.iters == 0 and not torch.any(x).item()


def test_bicgstab_reports_no_convergence():
    from paper_1811_11992_amd import isc
    wl, m, Jd, b = _system("C1", 22)
    c = isc.Context(wl)
    x, info, st = c.isc_solve_bicgstab(_dev(Jd), _dev(b), max_iters=2, rtol=1e-8, check=False)
    assert st == isc.ISC_ERR_LINEAR_NOCONV and info.iters == 2
    assert info.relres_true > 1e-8 and np.isfinite(info.relres_true)


def test_bicgstab_breakdown_restarts_a_bounded_number_of_times():
    """The oracle pin's breakdown system (b^T A M^-1 b = 0, so (r~, v) = 0 at the
    first iteration) on the GPU: the same bounded restarts and the same error,
    x left at zero; a nearby right-hand side converges."""
    from test_oracle_pins import _synthetic_decoupled, _bicgstab_breakdown_rhs
    from paper_1811_11992_amd import isc
    wl, m, Jd = _synthetic_decoupled("tiny:2x2x1", 4, 0.6)
    b = _bicgstab_breakdown_rhs(m, Jd)
    c = isc.Context(wl)
    x, info, st = c.isc_solve_bicgstab(_dev(Jd), _dev(b), max_iters=50, rtol=1e-8, check=False)
    assert st == isc.ISC_ERR_LINEAR_NOCONV and info.iters == 0 and info.restarts == 8
    assert np.all(_host(x) == 0.0)
    b2 = b + 1e-3 * np.random.default_rng(1).standard_normal(b.shape)
    x, info, st = c.isc_solve_bicgstab(_dev(Jd), _dev(b2), max_iters=200, rtol=1e-10)
    assert st == 0 and info.relres_true <= 1e-10
    r = b2 - m.spmv(Jd, _host(x))
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b2)


def test_bicgstab_inside_the_newton_step_reaches_the_oracle_roots():
    """Five implicit C1 steps with BiCGSTAB as the Krylov method of
    isc_newton_step reach the roots of the oracle's BILU(0)-GMRES run (both
    in parity mode), step sizes equal."""
    from test_gpu_parity import _drive
    from paper_1811_11992_amd import isc
    wl = I.make_workload("C1")
    m = O.Model(wl)
    nsteps = 5

    def o_step(u, uo, dt, tol):
        st, v, info = m.newton_step(u, uo, dt, tol=tol)
        u[...] = v
        return st, bool(info.converged)

    hist_o, dts_o = _drive(o_step, lambda a: np.array(a, copy=True), wl.u0, wl.dt, nsteps)
    c = isc.Context(wl)
    lin = isc.bicgstab_opts()

    def g_step(u, uo, dt, tol):
        st, info = c.isc_newton_step(u, uo, dt, tol=tol, lin=lin)
        assert info.lin.iters >= 0
        return st, bool(info.converged)

    hist_g, dts_g = _drive(g_step, lambda a: _dev(a) if isinstance(a, np.ndarray) else a.clone(), wl.u0, wl.dt,
                           nsteps)
    assert dts_g == dts_o
    floor = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 5000.0])
    for s in range(nsteps):
        torch.cuda.synchronize()
        ug = hist_g[s + 1].cpu().numpy()
        rel = np.abs(ug - hist_o[s + 1]).max(axis=1) / np.maximum(np.abs(hist_o[s + 1]).max(axis=1), floor)
        assert np.all(rel <= 1e-9), (s, rel)


def test_isc_solve_selects_bicgstab():
    """isc_solve with ISC_KRYLOV_BICGSTAB is isc_solve_bicgstab with
    restart x max_restarts iterations; the other precisions and
    preconditioners refuse it."""
    from paper_1811_11992_amd import isc
    wl, m, Jd, b = _system("tiny:9x17x6", 5)
    c = isc.Context(wl)
    x1, i1, st1 = c.isc_solve(_dev(Jd), _dev(b), isc.bicgstab_opts(rtol=1e-10))
    x2, i2, st2 = c.isc_solve_bicgstab(_dev(Jd), _dev(b), max_iters=600, rtol=1e-10)
    assert st1 == 0 and st2 == 0 and i1.iters == i2.iters
    assert torch.equal(x1, x2)
    bad = isc.solve_opts(precision=isc.ISC_MIXED, inner_iters=4, krylov=isc.ISC_KRYLOV_BICGSTAB)
    _, _, st3 = c.isc_solve(_dev(Jd), _dev(b), bad, check=False)
    assert st3 == isc.ISC_ERR_ARG
