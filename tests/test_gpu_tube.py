"""The combustion tube of Section 4.1 (12 cells, heater ignition, air
injected at the top, production at the bottom) on the GPU against the oracle,
step by step through the heating period and beyond: both sides take the same
step sizes, their states agree to 1e-9 per variable (floors 1 Pa, 1 K, 1,
C_cmax) after every step, and the oracle's scaled residual at every GPU root
is <= 1e-10 or, where that is below what the state can resolve, within a few
times the rounding floor of the residual (sum over a row's Jacobian entries
of |dF/du| times the spacing of the floating-point numbers at u, scaled like
the residual): in the tube's small, 12.7-darcy cells the energy rows change
by about 0.5 W per pascal through the gas convection, so one unit in the last
place of the pressure (2e-9 Pa) moves them by about 1e-9 W, 2.6e-10 of their
scale.  The run ignites the top cell (checked against the oracle's own tube
test).  Both sides run in parity mode: Newton to 1e-10, then one more
iteration."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1811_11992_amd import inputs as I

pytestmark = pytest.mark.gpu

FLOOR = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 5000.0])


def _scaled_residual_and_floor(m, wl, u, uo, dt):
    """The oracle's scaled residual at u and the rounding floor of that
    quantity (one ulp of every unknown through the Jacobian's row sums)."""
    fl = m.fluid
    F, J = m.assemble(u, uo, dt)
    V = wl.dx * wl.dy * wl.dz
    sm = V * wl.poro * fl.rho_ref[0] / dt
    se = V * (1.0 - wl.poro) * fl.cp_rock / dt
    scale = np.where(np.arange(8)[None, :] == 6, se[:, None], sm[:, None])
    ulp = np.spacing(np.abs(u))                          # [8][N]
    floor = np.zeros((m.n, 8))
    for i in range(m.n):
        for b in range(m.row_ptr[i], m.row_ptr[i + 1]):
            floor[i] += np.abs(J[b]) @ ulp[:, m.col_idx[b]]
    return float((np.abs(F) / scale).max()), float((floor / scale).max())


def _run(step_fn, set_heater, copy, wl, nsteps):
    u = copy(wl.u0)
    t = 0.0
    h = wl.heater
    hist, dts = [copy(u)], []
    for _ in range(nsteps):
        set_heater(h["cell"], h["rate_W"] if t < h["stop_s"] else 0.0)
        uo = copy(u)
        dt = wl.dt
        for _cut in range(5):
            u = copy(uo)
            ok = False
            for _k in range(13):
                st, conv = step_fn(u, uo, dt, 1e-10)
                if st != 0:
                    break
                if conv:
                    ok = True
                    break
            if ok:
                st, _ = step_fn(u, uo, dt, 0.0)
                assert st == 0
                break
            dt *= 0.5
        assert ok
        t += dt
        hist.append(copy(u))
        dts.append(dt)
    return hist, dts


@pytest.mark.parametrize("precond", ["bilu0", "cpr"])
def test_tube_run_matches_oracle_per_step(precond):
    from paper_1811_11992_amd import isc
    wl = I.make_workload("TUBE")
    m = O.Model(wl)

    def o_step(u, uo, dt, tol):
        st, v, info = m.newton_step(u, uo, dt, tol=tol)
        u[...] = v
        return st, bool(info.converged)

    hist_o, dts_o = _run(o_step, m.set_heater, lambda a: np.array(a, copy=True), wl, wl.nsteps)
    c = isc.Context(wl, cpr_p_iters=6 if precond == "cpr" else None)
    lin = isc.cpr_opts(p_iters=6) if precond == "cpr" else isc.solve_opts()

    def g_step(u, uo, dt, tol):
        st, info = c.isc_newton_step(u, uo, dt, tol=tol, lin=lin)
        return st, bool(info.converged)

    def dev(a):
        return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")

    hist_g, dts_g = _run(g_step, c.isc_set_heater, lambda a: dev(a) if isinstance(a, np.ndarray) else a.clone(),
                         wl, wl.nsteps)
    assert dts_g == dts_o
    worst = 0.0
    for s in range(wl.nsteps):
        ug = hist_g[s + 1].cpu().numpy()
        rel = np.abs(ug - hist_o[s + 1]).max(axis=1) / np.maximum(np.abs(hist_o[s + 1]).max(axis=1), FLOOR)
        worst = max(worst, rel.max())
        assert np.all(rel <= 1e-9), (s, rel)
        t_start = sum(dts_g[:s])
        h = wl.heater
        m.set_heater(h["cell"], h["rate_W"] if t_start < h["stop_s"] else 0.0)
        res, floor = _scaled_residual_and_floor(m, wl, ug, hist_g[s].cpu().numpy(), dts_g[s])
        assert res <= max(1e-10, 8 * floor), (s, res, floor)
    ug = hist_g[-1].cpu().numpy()
    print(f"tube ({precond}): {wl.nsteps} steps, {sum(dts_g):.0f} s, top cell {ug[I.T, 0]:.1f} K, "
          f"largest state difference to the oracle {worst:.1e}", flush=True)
    assert ug[I.T, 0] > 550.0
