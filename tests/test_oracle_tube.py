"""The combustion tube of Section 4.1 on the oracle (CPU): the heater enters
the energy balance of its cell and nothing else, and the 12-cell tube, heated
at the top for its first 30 minutes while air is injected, ignites: the top
cell passes 550 K, its oxygen is consumed, coke forms there, and the
producer at the bottom produces.  The paper's comparison with CMG STARS
(its tube figures) cannot be repeated without the STARS curves, so the
tube's physics beyond these checks is parity unpinned."""
import numpy as np

import oracle as O
from paper_1811_11992_amd import inputs as I


def tube_run(m, wl, nsteps, tol=1e-10):
    """Implicit steps of the tube with its heater schedule (on while the
    step starts before the stop time); a failed Newton iteration halves the
    step.  Returns the states after each step and the step sizes."""
    u = wl.u0.copy()
    t = 0.0
    hist, dts = [u.copy()], []
    h = wl.heater
    for _ in range(nsteps):
        m.set_heater(h["cell"], h["rate_W"] if t < h["stop_s"] else 0.0)
        uo = u.copy()
        dt = wl.dt
        for _cut in range(5):
            u = uo.copy()
            ok = False
            for _k in range(13):
                st, u, info = m.newton_step(u, uo, dt, tol=tol)
                if st != 0:
                    break
                if info.converged:
                    ok = True
                    break
            if ok:
                break
            dt *= 0.5
        assert ok
        t += dt
        hist.append(u.copy())
        dts.append(dt)
    return hist, dts


def test_heater_enters_the_energy_balance_of_its_cell_only():
    wl = I.make_workload("TUBE")
    m = O.Model(wl)
    u = I.random_states(wl, 3)
    F0 = m.residual(u, wl.u0, wl.dt)
    m.set_heater(4, 123.25)
    F1 = m.residual(u, wl.u0, wl.dt)
    d = F1 - F0
    assert d[4, 6] == -123.25
    d[4, 6] = 0.0
    assert np.all(d == 0.0)
    W, R = m.sources(u)
    m.set_heater(-1, 0.0)
    W0, R0 = m.sources(u)
    assert W[4, 6] - W0[4, 6] == 123.25 and np.array_equal(R, R0)


def test_tube_ignites_under_its_heater():
    wl = I.make_workload("TUBE")
    m = O.Model(wl)
    hist, dts = tube_run(m, wl, wl.nsteps)
    u = hist[-1]
    assert sum(dts) > wl.heater["stop_s"]
    assert u[I.T, 0] > 550.0                          # the heated top cell is burning
    assert u[I.YO2, 0] < 0.05 < wl.u0[I.YO2, 0]       # its oxygen is consumed
    assert u[I.CC, 0] > 100.0                         # coke deposited there
    assert u[I.T, -1] < 320.0                         # the front has not reached the bottom
    # the bottom cell stays above the producer's bottom-hole pressure: it produces
    assert np.all(np.array([h[I.P, -1] for h in hist[1:]]) > wl.wells[1]["target"])
