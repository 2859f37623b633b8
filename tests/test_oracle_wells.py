"""Pins of the oracle's controlled wells (bottom-hole pressure as an unknown,
well-modelling subsection of Section 2.2 and the last row of the table of
unknowns and equations).

What fixes each check, independently of the code under test:
  * a well under BHP control is the fixed-BHP local source the oracle already
    pins: the same Newton roots, step by step;
  * the well rows B = dF/dbhp, C = dR/du, D = dR/dbhp are derivatives: central
    finite differences of the residual and of the well equation;
  * a rate-controlled well delivers its target, with the phase rates
    recomputed here from the Peaceman formula WI rho_a k_ra / mu_a (bhp - p)
    out of the oracle's per-cell densities, relative permeabilities and
    viscosities -- for every phase mask and for the injector;
  * eliminating the well rows (Schur complement, GMRES) gives the solution
    of the full bordered Newton system, solved densely here;
  * the switching rules: a rate the limit cannot deliver ends on the limit,
    and the way back is taken at the next step's start.
"""
import copy

import numpy as np
import pytest

import oracle as O
from paper_1811_11992_amd import inputs as I

D = O.DIAG


def _model(wl):
    return O.Model(wl)


def _run(m, wl, nsteps):
    st, u, recs, hist = m.run(wl.u0.copy(), wl.dt, nsteps, keep_history=True)
    assert st == nsteps, st
    return u, recs, hist


def _cw(dims="8x6x4", prod=None, inj=None):
    wl = I.make_workload("CW:" + dims)
    if prod:
        wl.wells[1].update(prod)
    if inj:
        wl.wells[0].update(inj)
    return wl


def _phase_rates(m, u, wells):
    """Per controlled well: per-perforation phase molar rates Q[k][a] (Q < 0
    produced) recomputed from the Peaceman formula and the per-cell
    densities, relative permeabilities and viscosities."""
    dg = m.diag(u)
    cells, kinds, wi, _ = m.perf_info()
    bhp, _ = m.well_state()
    out = []
    p0, w = 0, 0
    for wd in wells:
        npf = len(wd["cells"])
        if wd["kind"] not in (I.WELL_PRODUCER, I.WELL_INJECTOR):
            p0 += npf
            continue
        Q = np.zeros((npf, 3))
        for k in range(npf):
            i = cells[p0 + k]
            lam = [dg[i, D["krw"] + a] * dg[i, D["rho_w"] + a] / dg[i, D["mu_w"] + a] for a in range(3)]
            p = u[0, i]
            if wd["kind"] == I.WELL_PRODUCER and p > bhp[w]:
                Q[k] = [wi[p0 + k] * lam[a] * (bhp[w] - p) for a in range(3)]
            elif wd["kind"] == I.WELL_INJECTOR and bhp[w] > p:
                Q[k, 0] = wi[p0 + k] * sum(lam) * (bhp[w] - p)   # total, carried in column 0
        out.append(Q)
        p0 += npf
        w += 1
    return out


def test_bhp_control_is_the_local_source_producer():
    wl = I.make_workload("C1")
    u1, r1, h1 = _run(_model(wl), wl, 5)
    wl2 = copy.deepcopy(wl)
    wl2.wells[1] = dict(kind=I.WELL_PRODUCER, cells=wl.wells[1]["cells"], target=I.P0, control=I.CTRL_BHP)
    m2 = _model(wl2)
    u2, r2, h2 = _run(m2, wl2, 5)
    assert [r["cuts"] for r in r1] == [r["cuts"] for r in r2]
    for s in range(6):
        rel = np.abs(h2[s] - h1[s]).max(axis=1) / np.maximum(np.abs(h1[s]).max(axis=1), 1e-30)
        assert np.all(rel <= 1e-12), (s, rel)
    assert m2.well_state()[0][0] == I.P0


@pytest.mark.parametrize("ctrl", [I.CTRL_TOTAL, I.CTRL_OIL, I.CTRL_WATER, I.CTRL_GAS, I.CTRL_LIQUID])
def test_fixed_rate_well_returns_its_rate(ctrl):
    """Water/oil/gas/liquid/total rate control of the producer and the
    injector's total rate, each met to rounding at every converged step."""
    wl = _cw(prod=dict(control=ctrl, target=0.3 * I.make_workload("CW:8x6x4").wells[0]["target"]))
    m = _model(wl)
    u = wl.u0.copy()
    for s in range(3):
        st, u, recs, _ = m.run(u, wl.dt, 1)
        assert st == 1
        bhp, on = m.well_state()
        Qi, Qp = _phase_rates(m, u, wl.wells)
        # injector: total injected = target (its limit is far)
        assert on[0] == 0
        assert abs(Qi[:, 0].sum() - wl.wells[0]["target"]) <= 1e-9 * wl.wells[0]["target"]
        # producer: the phases in the mask
        mask = [a for a in range(3) if ctrl & (1 << a)]
        if on[1] == 0:
            q = -Qp[:, mask].sum()
            assert abs(q - wl.wells[1]["target"]) <= 1e-9 * wl.wells[1]["target"], (s, q)
            assert bhp[1] >= wl.wells[1]["limit"]
        else:
            assert bhp[1] == wl.wells[1]["limit"]
        # the source terms carry the same phase rates: total moles over rows 0..5
        W = np.zeros((m.n, 8))
        O.lib().orc_sources(m.h, O._p(np.ascontiguousarray(u)), O._p(W), None)
        prod_cells = wl.wells[1]["cells"]
        assert abs(W[prod_cells, :6].sum() - Qp.sum()) <= 1e-12 * abs(Qp).sum() + 1e-300
        inj_cells = wl.wells[0]["cells"]
        zsum = sum(I.AIR[:6])
        assert abs(W[inj_cells, :6].sum() - Qi[:, 0].sum() * zsum) <= 1e-12 * abs(Qi).sum()


def _border_state(ctrl, nsteps=2):
    q = I.make_workload("CW:5x4x3").wells[0]["target"]
    wl = _cw("5x4x3", prod=dict(control=ctrl, target=0.05 * q))
    m = _model(wl)
    u, _, _ = _run(m, wl, nsteps)
    return wl, m, u


@pytest.mark.parametrize("ctrl", [I.CTRL_TOTAL, I.CTRL_OIL, I.CTRL_GAS])
def test_well_rows_are_the_derivatives(ctrl):
    wl, m, u = _border_state(ctrl)
    bhp, on = m.well_state()
    assert not on.any()
    R, Dd, B, C = m.well_border(u)
    uo = u.copy()
    dt = wl.dt
    p0 = 0
    for w, wd in enumerate(wl.wells):
        cells = wd["cells"]
        h = min(1e-7 * bhp[w], 0.01 * np.abs(u[0, cells] - bhp[w]).min())   # no perforation changes side
        assert h > 1e-3
        # B = dF/dbhp and D = dR/dbhp
        Fp, Fm = [], []
        for sgn, store in ((1, Fp), (-1, Fm)):
            b = bhp.copy()
            b[w] += sgn * h
            m.set_well_state(b, on)
            store.append(m.residual(u, uo, dt))
            store.append(m.well_border(u)[0][w])
        m.set_well_state(bhp, on)
        dF = (Fp[0] - Fm[0]) / (2 * h)
        for k, i in enumerate(cells):
            scale = np.abs(B[p0 + k]).max()
            assert np.all(np.abs(dF[i] - B[p0 + k]) <= 1e-6 * scale + 1e-300), (w, k, dF[i], B[p0 + k])
        others = np.setdiff1d(np.arange(m.n), cells)
        assert np.abs(dF[others]).max() == 0.0
        assert abs((Fp[1] - Fm[1]) / (2 * h) - Dd[w]) <= 1e-6 * abs(Dd[w])
        # C = dR/du at the perforated cells
        for k, i in enumerate(cells):
            for v in range(8):
                hv = 1e-6 * max(abs(u[v, i]), {0: 1e5, 4: 100.0, 7: 100.0}.get(v, 1e-3))
                up, um = u.copy(), u.copy()
                up[v, i] += hv
                um[v, i] -= hv
                fd = (m.well_border(up)[0][w] - m.well_border(um)[0][w]) / (2 * hv)
                tol = 1e-5 * np.abs(C[p0 + k] * np.maximum(np.abs(u[:, i]), 1e-3)).max() / max(abs(u[v, i]), 1e-3)
                assert abs(fd - C[p0 + k, v]) <= tol + 1e-300, (w, k, v, fd, C[p0 + k, v])
        p0 += len(cells)


@pytest.mark.parametrize("case", ["rates", "bhp_off_target"])
def test_schur_elimination_solves_the_bordered_system(case):
    """One Newton iteration near a root: the oracle's update of (u, bhp)
    equals the dense solution of [J B; C D] [du; dbhp] = -[F; R] (no step
    limit active).  "rates": both wells on a rate, the targets moved a little
    (R ~ 0 after the well-line solve); "bhp_off_target": the producer under
    BHP control with its bhp 2% of P0 away from the target, so that R != 0."""
    wl = _cw("4x3x2")
    m = _model(wl)
    u, _, _ = _run(m, wl, 2)
    uo = u.copy()
    bhp, on = m.well_state()
    wl2 = copy.deepcopy(wl)
    wl2.wells[0]["target"] *= 1.02
    if case == "rates":
        wl2.wells[1]["target"] *= 0.98
    else:
        wl2.wells[1].update(control=I.CTRL_BHP, target=float(bhp[1]) + 0.02 * I.P0)
    m3 = _model(wl2)
    m3.set_well_state(bhp, on)
    m3.well_solve(u)                 # what the Newton iteration does first
    bhp = m3.well_state()[0]
    F, Jb = m3.assemble(u, uo, wl.dt)
    R, Dd, B, C = m3.well_border(u)
    if case == "bhp_off_target":
        assert abs(R[1] + 0.02 * I.P0) <= 1e-6 and Dd[1] == 1.0 and not C[wl.nz:].any()
    n = m3.n
    Jd = np.zeros((8 * n, 8 * n))
    for i in range(n):
        for b in range(m3.row_ptr[i], m3.row_ptr[i + 1]):
            j = m3.col_idx[b]
            Jd[8 * i:8 * i + 8, 8 * j:8 * j + 8] = Jb[b]
    nw = len(R)
    A = np.zeros((8 * n + nw, 8 * n + nw))
    A[:8 * n, :8 * n] = Jd
    p0 = 0
    for w, wd in enumerate(wl2.wells):
        for k, i in enumerate(wd["cells"]):
            A[8 * i:8 * i + 8, 8 * n + w] = B[p0 + k]
            A[8 * n + w, 8 * i:8 * i + 8] = C[p0 + k]
        A[8 * n + w, 8 * n + w] = Dd[w]
        p0 += len(wd["cells"])
    rhs = -np.concatenate([F.reshape(-1), R])
    x = np.linalg.solve(A, rhs)
    du = x[:8 * n].reshape(n, 8)
    st, u_new, info = m3.newton_step(u, uo, wl.dt, rtol=1e-14, max_restarts=200)
    assert st == 0 and not info.converged
    got = (u_new - u).T
    # cells where the update's safeguards (step limits, saturation and
    # fraction rules) act are left out
    v = u.T + du
    so = 1.0 - v[:, 5] - v[:, 6]
    free = ((v[:, 1:4] >= 0) & (v[:, 1:4] <= 1)).all(axis=1) & (v[:, 5:8] >= 0).all(axis=1) & (so >= 0)
    free &= np.abs(du[:, 0]) <= 0.2 * np.abs(u[0])
    assert free.sum() >= n // 2
    scale = np.abs(du[free]).max(axis=0) + 1e-300
    err = np.abs(got[free] - du[free]).max(axis=0)
    assert np.all(err <= 1e-7 * scale), err / scale
    bhp_new, _ = m3.well_state()
    assert np.allclose(bhp_new - bhp, x[8 * n:], rtol=1e-7, atol=1e-9 * abs(bhp).max())


def test_unreachable_rate_ends_on_the_limit_and_returns_at_a_step_start():
    wl = _cw(prod=dict(target=50.0, limit=0.97 * I.P0))   # far above what 0.97 P0 delivers
    m = _model(wl)
    u, recs, hist = _run(m, wl, 3)
    bhp, on = m.well_state()
    assert on[1] == 1 and bhp[1] == wl.wells[1]["limit"]
    q = -_phase_rates(m, u, wl.wells)[1].sum()
    assert q < wl.wells[1]["target"]
    # a lower target is reachable at the limit: the next step's start returns
    wl3 = copy.deepcopy(wl)
    wl3.wells[1]["target"] = 0.5 * q
    m3 = _model(wl3)
    m3.set_well_state(bhp, on)
    assert m3.well_controls(u) == 1
    assert m3.well_state()[1][1] == 0
    # and it holds within a step: a Newton iteration does not leave the limit
    m.set_well_state(bhp, on)
    uo = u.copy()
    st, u2, info = m.newton_step(u, uo, wl.dt)
    assert m.well_state()[1][1] == 1


def test_injector_limit():
    wl = _cw(inj=dict(target=50.0, limit=I.P0 + 2.0e5))
    m = _model(wl)
    _run(m, wl, 2)
    bhp, on = m.well_state()
    assert on[0] == 1 and bhp[0] == I.P0 + 2.0e5


def test_adjoint_refuses_controlled_wells():
    wl = _cw("4x3x2")
    m = _model(wl)
    g_logk = np.zeros(m.n)
    g_A = np.zeros(4)
    st, _ = m.adjoint_step(wl.u0, wl.u0, wl.dt, None, wl.dt, g_logk, g_A)
    assert st == -2


def test_switching_thresholds():
    """Held at its limit, a well returns to its rate exactly when the limit
    would move more than the target: a target 1% above what the limit
    delivers keeps it there, 1% below sends it back."""
    wl = _cw(prod=dict(target=50.0, limit=0.97 * I.P0))
    m = _model(wl)
    u, _, _ = _run(m, wl, 2)
    bhp, on = m.well_state()
    assert on[1] == 1
    q = -_phase_rates(m, u, wl.wells)[1].sum()
    for factor, back in ((1.01, 0), (0.99, 1)):
        wl3 = copy.deepcopy(wl)
        wl3.wells[1]["target"] = factor * q
        m3 = _model(wl3)
        m3.set_well_state(bhp, on)
        assert m3.well_controls(u) == back
        assert m3.well_state()[1][1] == 1 - back


def test_well_rows_count_in_the_convergence_test():
    """The scaled residual of the well rows, by hand: a rate row by
    V phi rho_ref,W / dt of its first perforated cell, a BHP row by the
    pressure held; a converged state whose BHP well is off its target is
    not converged, by exactly that amount."""
    wl = _cw("4x3x2", prod=dict(control=I.CTRL_BHP, target=0.95 * I.P0))
    m = _model(wl)
    u, _, hist = _run(m, wl, 1)
    uo = hist[0]
    V = wl.dx * wl.dy * wl.dz
    fl = I.physics_card()
    s_rate = V * wl.poro[wl.wells[0]["cells"][0]] * fl.rho_ref[0] / wl.dt
    assert m.well_scaled_norm([3.0 * s_rate, 0.0], wl.dt) == pytest.approx(3.0, rel=1e-14)
    assert m.well_scaled_norm([0.0, -0.01 * 0.95 * I.P0], wl.dt) == pytest.approx(0.01, rel=1e-14)
    bhp, on = m.well_state()
    st, _, info = m.newton_step(u, uo, wl.dt)   # the step's root
    assert st == 0 and info.converged
    # the same state against a BHP target moved by 1e-8: the cells still
    # balance, the well row alone is off
    wl2 = copy.deepcopy(wl)
    wl2.wells[1]["target"] = 0.95 * I.P0 * (1 + 1e-8)
    m2 = _model(wl2)
    m2.set_well_state(bhp, on)
    assert m2.scaled_norm(m2.residual(u, uo, wl.dt), wl.dt) <= 1e-10
    st, _, info = m2.newton_step(u, uo, wl.dt)
    assert st == 0 and not info.converged
    assert info.res_scaled == pytest.approx(1e-8, rel=1e-6)
