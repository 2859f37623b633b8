"""Differentiation form on the GPU: isc_adjoint against the oracle's reference
adjoint on identical states, the autograd gradient against finite
differences of GPU forward runs, and checkpointing invariance.

Tolerances: adjoint states and gradients within 1e-7 (relative to their
largest entries) of the oracle (both solve the transposed systems to
1e-12..1e-13); gradient directional derivatives within 1e-6 of
Richardson-extrapolated central differences."""
import numpy as np
import pytest
import torch

from paper_1811_11992_amd import inputs as I
import oracle as O

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def oracle_forward(m, wl, nsteps, dt):
    u = wl.u0.copy()
    hist = [u.copy()]
    for _ in range(nsteps):
        uo = u.copy()
        for _k in range(14):
            st, u, info = m.newton_step(u, uo, dt, tol=1e-10)
            assert st == 0
            if info.converged:
                break
        assert info.converged
        st, u, _ = m.newton_step(u, uo, dt, tol=0.0)
        hist.append(u.copy())
    return hist


def _compare_adjoint(name, nsteps, dtfac):
    from paper_1811_11992_amd import isc
    wl = I.make_workload(name)
    dt = wl.dt * dtfac
    m = O.Model(wl)
    hist = oracle_forward(m, wl, nsteps, dt)
    c = isc.Context(wl)
    go, gAo = np.zeros(m.n), np.zeros(4)
    gg = torch.zeros(m.n, dtype=torch.float64, device="cuda")
    gAg = [0.0] * 4
    lam_o, lam_g = None, None
    for n in range(nsteps, 0, -1):
        st, lo = m.adjoint_step(hist[n], hist[n - 1], dt, lam_o, dt, go, gAo)
        assert st == 0
        lg = torch.empty((m.n, 8), dtype=torch.float64, device="cuda")
        gAg, info = c.isc_adjoint(dev(hist[n]), dev(hist[n - 1]), dt, lam_g, dt, lg, gg, gAg)
        lgh = lg.cpu().numpy()
        scale = np.abs(lo).max(axis=0) + 1e-300
        assert np.all(np.abs(lgh - lo).max(axis=0) <= 1e-7 * scale.max()), (n, np.abs(lgh - lo).max(axis=0) / scale)
        lam_o, lam_g = lo, lg
    ggh = gg.cpu().numpy()
    assert np.abs(ggh - go).max() <= 1e-7 * np.abs(go).max()
    assert np.all(np.abs(np.array(gAg) - gAo) <= 1e-7 * np.abs(gAo).max())
    return go, gAo


@pytest.mark.parametrize("name,nsteps,dtfac", [("tiny:4x3x2", 3, 0.2), ("tiny:6x5x3", 2, 0.5)])
def test_adjoint_steps_match_oracle(name, nsteps, dtfac):
    _compare_adjoint(name, nsteps, dtfac)


def test_autograd_gradient_matches_finite_differences_and_checkpointing():
    from paper_1811_11992_amd import isc
    from paper_1811_11992_amd.adjoint import OilProduction, log_frequency_factors
    wl = I.make_workload("tiny:4x3x2")
    dt = wl.dt * 0.2
    nsteps = 4
    fl = I.physics_card()
    c = isc.Context(wl, fluid=fl)
    u0 = dev(wl.u0)
    logk0 = torch.tensor(wl.logk, dtype=torch.float64, device="cuda")
    lnA0 = log_frequency_factors(fl)
    grads = []
    for every in (1, 2):
        logk = logk0.clone().requires_grad_(True)
        lnA = lnA0.clone().requires_grad_(True)
        J = OilProduction.apply(logk, lnA, c, u0, dt, nsteps, every)
        J.backward()
        grads.append((logk.grad.cpu().numpy().copy(), lnA.grad.numpy().copy(), float(J)))
    # recomputed segments reproduce the stored states bitwise
    assert np.array_equal(grads[0][0], grads[1][0]) and np.array_equal(grads[0][1], grads[1][1])
    gk, gA, J0 = grads[0]

    def Jof(lk, la):
        with torch.no_grad():
            return float(OilProduction.apply(lk, la, c, u0, dt, nsteps, 5))

    rng = np.random.default_rng(3)
    for trial in range(3):
        vk = rng.standard_normal(wl.ncell)
        vA = rng.standard_normal(4) if trial else np.zeros(4)
        nrm = np.sqrt(vk @ vk + vA @ vA)
        vk, vA = vk / nrm, vA / nrm
        tk, tA = torch.tensor(vk, device="cuda"), torch.tensor(vA)

        def D(h):
            return (Jof(logk0 + h * tk, lnA0 + h * tA) - Jof(logk0 - h * tk, lnA0 - h * tA)) / (2 * h)

        h = 2e-4
        fd = (4 * D(h / 2) - D(h)) / 3
        ad = gk @ vk + gA @ vA
        scale = abs(ad) + 1e-3 * (np.abs(gk) @ np.abs(vk) + np.abs(gA) @ np.abs(vA))
        assert abs(fd - ad) <= 1e-6 * scale, (trial, fd, ad)
    # the oracle's reference adjoint on its own forward states gives the same gradient
    m = O.Model(wl, fl)
    hist = oracle_forward(m, wl, nsteps, dt)
    go, gAo = np.zeros(m.n), np.zeros(4)
    lam = None
    for n in range(nsteps, 0, -1):
        st, lam = m.adjoint_step(hist[n], hist[n - 1], dt, lam, dt, go, gAo)
    A = np.exp(lnA0.numpy())
    assert np.abs(gk - go).max() <= 1e-6 * np.abs(go).max()
    assert np.all(np.abs(gA - gAo * A) <= 1e-6 * np.abs(gAo * A).max())


def test_adjoint_on_the_60x60x10_grid_matches_oracle():
    """C4 grid (36,000 cells, 36,000 + 4 parameters), first step."""
    _compare_adjoint("C4", 1, 1.0)
