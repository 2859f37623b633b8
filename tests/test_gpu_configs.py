"""The configured workloads run as configured, against the oracle: the
sweeps' multi-brick static schedule on a grid with more bricks than
co-resident workgroups, the 60x60x10 FP64 run (three steps against the
oracle's states, fifty against the oracle's residual), three steps of the
2M-cell grid in FP64 and in the precision form (per-step error against the
FP64 run and the oracle's residual at both roots), the gradient of 20-step
cumulative oil production on the 60x60x10 grid against central differences
on 20 directions and against the oracle's adjoint at the last step, and a
state whose coke exceeds the limiter's bound.

Tolerances (per check): sweeps bitwise between schedules and <= 1e-10 of the
oracle's apply; states <= 1e-9 (FP64) / 1e-8 (precision form) per variable
with floors 1 Pa, 1 K, 1, C_cmax; the oracle's scaled residual at every root
<= 1e-10; directional derivatives within 1e-6 of Richardson-extrapolated
central differences; adjoint states within 1e-7 of the oracle's."""
import numpy as np
import pytest
import torch

from paper_1811_11992_amd import inputs as I
import oracle as O

pytestmark = pytest.mark.gpu

COL = np.array([1e6, 1.0, 1.0, 1.0, 100.0, 1.0, 1.0, 1000.0])
FLOOR = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 5000.0])


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _rel_states(a, b):
    return np.abs(a - b).max(axis=1) / np.maximum(np.abs(b).max(axis=1), FLOOR)


# --------------------------------------------------------------- sweeps, many bricks per workgroup
def test_sweeps_take_many_bricks_per_workgroup_and_match_oracle(monkeypatch):
    """100x100x20: 6,250 bricks of 4x4x2 cells, more than the device holds
    workgroups at once (at most eight 256-thread workgroups per compute unit),
    so under the static cooperative schedule every workgroup sweeps several
    bricks in turn.  z = M^-1 r of that schedule equals the one-launch-per-
    hyperplane schedule bit for bit and the oracle's apply to 1e-10; the fused
    sweep + SpMV gives the same z; the FP32 sweeps of the precision form give
    bitwise the same solve under both schedules."""
    from paper_1811_11992_amd import isc
    wl = I.make_workload("tiny:100x100x20")
    nbrick = (wl.nx // 4) * (wl.ny // 4) * (wl.nz // 2)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert nbrick > 8 * cus, (nbrick, cus)
    m = O.Model(wl)
    F, J = m.assemble(wl.u0, wl.u0, wl.dt)
    st, Jd, Fd, _ = m.decouple(J, F)
    assert st == 0
    st, LU, Dinv_o = m.bilu0(Jd)
    assert st == 0
    rng = np.random.default_rng(5)
    r = rng.standard_normal((m.n, 8))
    z_o = m.bilu0_apply(LU, Dinv_o, r)
    # the FP32 factor is formed in FP64 arithmetic from the FP32-rounded blocks
    Jd32 = Jd.astype(np.float32).astype(np.float64)
    st, LU32, Dinv32 = m.bilu0(Jd32)
    z32_o = m.bilu0_apply(LU32, Dinv32, r)
    out = {}
    for level in ("0", "1"):
        monkeypatch.setenv("ISC_LEVEL_SWEEPS", level)
        c = isc.Context(wl, inner_iters=12)
        Jg = dev(Jd)
        D = c.isc_bilu0(Jg)
        z = c.isc_bilu0_apply(Jg, D, dev(r))
        zf, wf = c.isc_bilu0_apply_spmv(Jg, D, dev(r))
        z32, w32 = c.isc_bilu0_apply_spmv32(Jg, dev(r))
        x, info, st = c.isc_solve(Jg, dev(-Fd), isc.solve_opts(precision=isc.ISC_MIXED, inner_iters=12, rtol=1e-8))
        assert st == 0 and info.relres_true <= 1e-8
        out[level] = (host(z), host(zf), host(z32), host(w32), host(x), info.iters, info.inner_iters_total)
        c.close()
    z_s, zf_s, z32_s, w32_s, x_s, it_s, in_s = out["0"]
    z_l, zf_l, z32_l, w32_l, x_l, it_l, in_l = out["1"]
    # FP64: bitwise across schedules and fused/separate, 1e-10 of the oracle
    assert np.array_equal(z_s, z_l) and np.array_equal(zf_s, z_s) and np.array_equal(zf_l, z_l)
    err = np.abs(z_s - z_o).max(axis=0)
    assert np.all(err <= 1e-10 * (np.abs(z_o).max(axis=0) + 1e-300)), err / np.abs(z_o).max(axis=0)
    # FP32 storage: against the oracle's FP64 apply of the same FP32-rounded
    # factor within the rounding of FP32 storage, under both schedules (the
    # per-hyperplane schedule forms its L D^-1 blocks from the FP32 copy, the
    # sync-free factor rounds FP64 products, so the two differ by rounding)
    for z32 in (z32_s, z32_l):
        err32 = (np.abs(z32 - z32_o).max(axis=0) / (np.abs(z32_o).max(axis=0) + 1e-300)).max()
        print(f"FP32 apply vs the oracle's FP64 apply of the FP32-rounded factor: {err32:.2e}", flush=True)
        assert err32 <= 1e-4
    d32 = (np.abs(z32_s - z32_l).max(axis=0) / (np.abs(z32_l).max(axis=0) + 1e-300)).max()
    print(f"FP32 apply, static vs per-hyperplane schedule: {d32:.2e}", flush=True)
    assert d32 <= 1e-5
    wo = m.spmv(Jd32, z32_s)
    bound = np.abs(z32_s) + m.spmv(np.abs(Jd32), np.abs(z32_s))
    assert np.all(np.abs(w32_s - wo) <= 1e-5 * bound.max(axis=0)[None, :])
    assert np.all(np.abs(w32_l - wo) <= 1e-5 * bound.max(axis=0)[None, :])
    # the whole precision-form solve: the same iteration counts under both schedules
    assert it_s == it_l and in_s == in_l
    print(f"mixed solve, {it_s} outer / {in_s} inner iterations under both schedules; solutions differ by "
          f"{(np.abs(x_s - x_l).max(axis=0) / np.abs(x_l).max(axis=0)).max():.1e}", flush=True)


# --------------------------------------------------------------- 60x60x10, FP64 BILU(0)-GMRES(30)
def test_c2_first_steps_match_oracle_and_fifty_steps_reach_its_roots():
    from test_gpu_parity import _drive
    from paper_1811_11992_amd import isc
    wl = I.make_workload("C2")
    m = O.Model(wl)
    c = isc.Context(wl)

    def o_step(u, uo, dt, tol):
        st, v, info = m.newton_step(u, uo, dt, tol=tol)
        u[...] = v
        return st, bool(info.converged)

    def g_step(u, uo, dt, tol):
        st, info = c.isc_newton_step(u, uo, dt, tol=tol)
        return st, bool(info.converged)

    n_par = 3
    hist_o, dts_o = _drive(o_step, lambda a: np.array(a, copy=True), wl.u0, wl.dt, n_par)
    hist_g, dts_g = _drive(g_step, lambda a: dev(a) if isinstance(a, np.ndarray) else a.clone(), wl.u0, wl.dt,
                           n_par)
    assert dts_g == dts_o
    for s in range(n_par):
        rel = _rel_states(host(hist_g[s + 1]), hist_o[s + 1])
        print(f"C2 step {s + 1}: max relative state difference to the oracle {rel.max():.2e}", flush=True)
        assert np.all(rel <= 1e-9), (s, rel)
    # the configured 50 steps (the first three above), each root checked by the oracle's residual
    sim = isc.Simulator(c, tol=1e-10)
    u = hist_g[-1].clone()
    worst, cuts = 0.0, 0
    for s in range(n_par, wl.nsteps):
        u_prev = u.clone()
        rec = sim.step(u, wl.dt)     # the time loop halves a step whose Newton iteration fails
        st, _ = c.isc_newton_step(u, u_prev, rec["dt"], tol=0.0)    # one more iteration at the root
        assert st == 0
        res = m.scaled_norm(m.residual(host(u), host(u_prev), rec["dt"]), rec["dt"])
        worst = max(worst, res)
        cuts += rec["cuts"]
        assert res <= 1e-10, (s, res)
    print(f"C2: {wl.nsteps} steps ({cuts} halved), largest scaled oracle residual at a GPU root {worst:.2e}",
          flush=True)


# --------------------------------------------------------------- 200x200x50, FP64 and the precision form
def _window_residual(wl, fl, u, uo, cells_sampled):
    from test_gpu_fullsize import _window
    V = wl.dx * wl.dy * wl.dz
    worst = 0.0
    for c in cells_sampled:
        sub, cells, local = _window(wl, c)
        m = O.Model(sub, fl)
        F = m.residual(u[:, cells], uo[:, cells], wl.dt)[local]
        sm = V * wl.poro[c] * fl.rho_ref[0] / wl.dt
        se = V * (1.0 - wl.poro[c]) * fl.cp_rock / wl.dt
        worst = max(worst, float((np.abs(F) / np.where(np.arange(8) == 6, se, sm)).max()))
    return worst


def test_c3_steps_precision_form_against_fp64_and_oracle():
    """Three implicit steps of the 2M-cell workload, FP64 and the precision
    form (FP32 inner iterations 12, as benchmarked) each advancing its own
    state: the per-step state difference is <= 1e-8 and the oracle's scaled
    residual rows around sampled cells (including cell 1, next to the ignited
    injector cell) at both roots <= 1e-10."""
    from test_gpu_fullsize import _samples
    from paper_1811_11992_amd import isc
    wl = I.make_workload("C3")
    fl = I.physics_card()
    ctx = isc.Context(wl, restart=30, inner_iters=12)
    # sampled cells away from the perforations (a window holds no well terms)
    cells = _samples(wl, k=16, seed=11) + [1, wl.nx * wl.ny * 25 + wl.nx + 1]
    lins = {"fp64": isc.solve_opts(rtol=1e-8),
            "mixed": isc.solve_opts(rtol=1e-8, precision=isc.ISC_MIXED, inner_iters=12)}
    states = {k: dev(wl.u0) for k in lins}
    for s in range(3):
        roots = {}
        for k, lin in lins.items():
            u = states[k]
            uo = u.clone()
            for it in range(14):
                st, info = ctx.isc_newton_step(u, uo, wl.dt, 1e-10, lin)
                assert st == 0, (k, s, it, st)
                if info.converged:
                    break
            assert info.converged, (k, s)
            st, info = ctx.isc_newton_step(u, uo, wl.dt, 0.0, lin)
            assert st == 0
            roots[k] = (host(u), host(uo))
        rel = _rel_states(roots["mixed"][0], roots["fp64"][0])
        res64 = _window_residual(wl, fl, *roots["fp64"], cells)
        resmx = _window_residual(wl, fl, *roots["mixed"], cells)
        print(f"C3 step {s + 1}: mixed vs FP64 state {rel.max():.2e}; oracle residual at the FP64 root "
              f"{res64:.2e}, at the mixed root {resmx:.2e}", flush=True)
        assert np.all(rel <= 1e-8), (s, rel)
        assert res64 <= 1e-10 and resmx <= 1e-10, (s, res64, resmx)


# --------------------------------------------------------------- 60x60x10 gradient, 20 steps
def test_c4_gradient_matches_central_differences_and_oracle_adjoint():
    """Gradient of 20-step cumulative oil production with respect to
    (ln k [36,000], ln A [4]), checkpoints every 5 steps, against
    Richardson-extrapolated central differences of GPU forward runs on 20
    random unit directions (seed 7), and the GPU's last adjoint step against
    the oracle's on the same states."""
    from paper_1811_11992_amd import isc
    from paper_1811_11992_amd.adjoint import OilProduction, log_frequency_factors, _solve_step
    wl = I.make_workload("C4")
    fl = I.physics_card()
    nsteps, every = 20, 5
    c = isc.Context(wl, fluid=fl)
    u0 = dev(wl.u0)
    logk0 = torch.tensor(wl.logk, dtype=torch.float64, device="cuda")
    lnA0 = log_frequency_factors(fl)
    logk = logk0.clone().requires_grad_(True)
    lnA = lnA0.clone().requires_grad_(True)
    J = OilProduction.apply(logk, lnA, c, u0, wl.dt, nsteps, every)
    J.backward()
    gk, gA = logk.grad.cpu().numpy(), lnA.grad.numpy()

    def Jof(lk, la):
        with torch.no_grad():
            return float(OilProduction.apply(lk, la, c, u0, wl.dt, nsteps, every))

    rng = np.random.default_rng(7)
    h = 2e-4
    # Each forward run reaches its root to the rounding floor, which leaves J
    # reproducible to about 2e-14 of |J| between neighbouring parameter
    # values; the extrapolated difference quotient carries up to 3 dJ / h of
    # that (dJ bounded by 1e-13 |J|).  Directions whose derivative is a small
    # fraction of |J| are therefore checked to that floor rather than to 1e-6.
    noise = 3 * 1e-13 * abs(float(J)) / h
    worst = 0.0
    for d in range(20):
        vk = rng.standard_normal(wl.ncell)
        vA = rng.standard_normal(4)
        nrm = np.sqrt(vk @ vk + vA @ vA)
        vk, vA = vk / nrm, vA / nrm
        tk, tA = torch.tensor(vk, device="cuda"), torch.tensor(vA)

        def D(hh):
            return (Jof(logk0 + hh * tk, lnA0 + hh * tA) - Jof(logk0 - hh * tk, lnA0 - hh * tA)) / (2 * hh)

        fd = (4 * D(h / 2) - D(h)) / 3
        ad = gk @ vk + gA @ vA
        scale = abs(ad) + 1e-3 * (np.abs(gk) @ np.abs(vk) + np.abs(gA) @ np.abs(vA))
        worst = max(worst, abs(fd - ad) / abs(ad))
        print(f"C4 direction {d}: adjoint {ad:.10e}, differences {fd:.10e}, relative {abs(fd - ad) / abs(ad):.1e}",
              flush=True)
        assert abs(fd - ad) <= max(1e-6 * scale, noise), (d, fd, ad)
    print(f"C4: 20 directions, largest relative difference adjoint vs central differences {worst:.2e} "
          f"(rounding floor of the differences {noise:.1e})", flush=True)
    # the last step's adjoint against the oracle's on the GPU's states
    c.isc_set_params(logk=logk0, A=np.exp(lnA0.numpy()))
    lin = isc.solve_opts()
    u = u0.clone()
    prev = None
    for n in range(nsteps):
        prev = u
        u = _solve_step(c, u, wl.dt, 1e-10, 12, lin)
    un, unm1 = host(u), host(prev)
    m = O.Model(wl, fl)
    go, gAo = np.zeros(m.n), np.zeros(4)
    st, lam_o = m.adjoint_step(un, unm1, wl.dt, None, wl.dt, go, gAo)
    assert st == 0
    gg = torch.zeros(m.n, dtype=torch.float64, device="cuda")
    lg = torch.empty((m.n, 8), dtype=torch.float64, device="cuda")
    gAg, info = c.isc_adjoint(u, prev, wl.dt, None, wl.dt, lg, gg, [0.0] * 4)
    lgh = host(lg)
    assert np.abs(lgh - lam_o).max() <= 1e-7 * np.abs(lam_o).max()
    assert np.abs(host(gg) - go).max() <= 1e-7 * np.abs(go).max()
    assert np.all(np.abs(np.array(gAg) - gAo) <= 1e-7 * np.abs(gAo).max())


# --------------------------------------------------------------- coke beyond the limiter bound
def test_assemble_matches_oracle_with_coke_above_its_limit():
    """A state in which a third of the cells hold more coke than C_cmax (the
    cracking rate's limiter is clamped to zero there) and the rest random."""
    from test_gpu_parity import row_scale, jac_rel_err
    from paper_1811_11992_amd import isc
    wl = I.make_workload("tiny:13x7x5")
    fl = I.physics_card()
    m = O.Model(wl, fl)
    c = isc.Context(wl, fluid=fl)
    u = I.random_states(wl, 909)
    uo = I.random_states(wl, 910)
    rng = np.random.default_rng(1)
    over = rng.choice(wl.ncell, wl.ncell // 3, replace=False)
    u[7, over] = fl.Ccmax * rng.uniform(1.05, 1.5, over.size)
    assert np.count_nonzero(m.diag(u)[over, O.DIAG["r0"] + 2]) == 0     # r3 = 0 where clamped
    Fo, Jo = m.assemble(u, uo, wl.dt)
    Fg, Jg = c.isc_assemble(dev(u), dev(uo), wl.dt)
    Fg, Jg = host(Fg), host(Jg)
    sc = row_scale(m, wl, u, uo, Fo)
    assert np.all(np.abs(Fg - Fo) <= 1e-12 * sc[None, :]), (np.abs(Fg - Fo) / sc).max()
    assert jac_rel_err(m, Jg, Jo) <= 1e-11
