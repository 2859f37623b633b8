"""GPU (libisc through its C-ABI) against the CPU oracle, element by element,
on identical seeded inputs.

Tolerances (stated per check):
  F            |dF| <= 1e-12 x (row scale: V/dt max|A_e| + max|F_e|)
  J blocks     <= 1e-11 x block-row max-norm, columns scaled by unit sizes
  C_L J, C_L F <= 1e-10 (same scaling), D^-1 <= 1e-10, SpMV/ILU apply <= 1e-10
  solve        true residual of the GPU solution (recomputed by the oracle)
               <= 1.01 rtol; distance to a tight oracle solution <= 1e-5
  Newton root  states within 1e-9 of the oracle's root (per-variable floors)
               and the oracle's scaled residual at the GPU root <= 1e-10
"""
import numpy as np
import pytest
import torch

from paper_1811_11992_amd import inputs as I
import oracle as O

pytestmark = pytest.mark.gpu

COL = np.array([1e6, 1.0, 1.0, 1.0, 100.0, 1.0, 1.0, 1000.0])   # unit size of each unknown
FLOOR = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 5000.0])   # state-comparison floors


def ctx_for(wl, **kw):
    from paper_1811_11992_amd import isc
    return isc.Context(wl, **kw)


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def row_scale(m, wl, u, uo, F):
    V = wl.dx * wl.dy * wl.dz
    a0 = O.DIAG["acc0"]
    acc = np.abs(m.diag(u)[:, a0:a0 + 8]).max(axis=0)
    acco = np.abs(m.diag(uo)[:, a0:a0 + 8]).max(axis=0)
    return V / wl.dt * np.maximum(acc, acco) + np.abs(F).max(axis=0) + 1e-300


def jac_rel_err(m, Jg, Jo, scale_rows=False):
    """max over block rows and equation rows of the row-relative block error,
    columns scaled by COL (and rows by 1/COL for decoupled blocks)"""
    worst = 0.0
    for i in range(m.n):
        b0, b1 = m.row_ptr[i], m.row_ptr[i + 1]
        A = Jo[b0:b1] * COL[None, None, :]
        B = Jg[b0:b1] * COL[None, None, :]
        if scale_rows:
            A = A / COL[None, :, None]
            B = B / COL[None, :, None]
        ref = np.abs(A).max(axis=(0, 2)) + 1e-300
        err = np.abs(A - B).max(axis=(0, 2))
        worst = max(worst, float((err / ref).max()))
    return worst


CASES = [("tiny:4x3x2", 101), ("tiny:13x7x5", 102), ("C1", None), ("C1", 103), ("tiny:1x1x6", 104)]


@pytest.mark.parametrize("name,seed", CASES)
def test_assemble_matches_oracle(name, seed):
    wl = I.make_workload(name)
    m = O.Model(wl)
    c = ctx_for(wl)
    if seed is None:
        u, uo = wl.u0, wl.u0
    else:
        u, uo = I.random_states(wl, seed), I.random_states(wl, seed + 1000)
    Fo, Jo = m.assemble(u, uo, wl.dt)
    Fg, Jg = c.isc_assemble(dev(u), dev(uo), wl.dt)
    Fg, Jg = host(Fg), host(Jg)
    sc = row_scale(m, wl, u, uo, Fo)
    assert np.all(np.abs(Fg - Fo) <= 1e-12 * sc[None, :]), (np.abs(Fg - Fo) / sc).max()
    assert jac_rel_err(m, Jg, Jo) <= 1e-11
    # run to run: bitwise identical
    Fg2, Jg2 = c.isc_assemble(dev(u), dev(uo), wl.dt)
    assert np.array_equal(host(Fg2), Fg) and np.array_equal(host(Jg2), Jg)


@pytest.mark.parametrize("dims", ["2x1x1", "1x1x2"])
def test_face_flux_is_bitwise_antisymmetric(dims):
    wl = I.make_workload("tiny:" + dims)
    wl.wells = []
    fl = I.physics_card(Afreq=(0.0, 0.0, 0.0, 0.0))
    c = ctx_for(wl, fluid=fl)
    u = I.random_states(wl, 7)
    F, J = c.isc_assemble(dev(u), dev(u), wl.dt)   # u_old = u: only the face flux remains
    F = host(F)
    assert np.array_equal(F[0], -F[1])


def _decoupled_case(name, seed):
    wl = I.make_workload(name)
    m = O.Model(wl)
    u = I.random_states(wl, seed)
    F, J = m.assemble(u, wl.u0, wl.dt)
    return wl, m, u, F, J


@pytest.mark.parametrize("name,seed", [("tiny:4x3x2", 5), ("tiny:13x7x5", 6), ("C1", 8)])
def test_decouple_matches_oracle(name, seed):
    wl, m, u, F, J = _decoupled_case(name, seed)
    c = ctx_for(wl)
    st, Jd, Fd, bad = m.decouple(J, F)
    assert st == 0
    Jg, Fg = dev(J), dev(F)
    st, badg = c.isc_decouple(Jg, Fg)
    assert st == 0 and badg == -1
    Jg, Fg = host(Jg), host(Fg)
    assert jac_rel_err(m, Jg, Jd, scale_rows=True) <= 1e-10
    a = Fd / COL
    b = Fg / COL
    ref = np.abs(a).max(axis=0) + 1e-300
    assert np.all(np.abs(a - b).max(axis=0) <= 1e-10 * ref)


def test_decouple_reports_singular_block():
    wl, m, u, F, J = _decoupled_case("tiny:4x3x2", 9)
    c = ctx_for(wl)
    bad_cell = 7
    dpos = [b for b in range(m.row_ptr[bad_cell], m.row_ptr[bad_cell + 1]) if m.col_idx[b] == bad_cell][0]
    J = J.copy()
    J[dpos, 3, :] = 0.0      # a zero equation row makes J_ii singular
    from paper_1811_11992_amd import isc
    st, badg = c.isc_decouple(dev(J), dev(F))
    assert st == isc.ISC_ERR_SINGULAR and badg == bad_cell
    st_o, _, _, bad_o = m.decouple(J, F)
    assert st_o == -4 and bad_o == bad_cell


@pytest.mark.parametrize("name,seed", [("tiny:4x3x2", 11), ("tiny:13x7x5", 12), ("C1", 13)])
def test_preconditioner_and_spmv_match_oracle(name, seed):
    wl, m, u, F, J = _decoupled_case(name, seed)
    st, Jd, Fd, _ = m.decouple(J, F)
    st, LU, Dinv_o = m.bilu0(Jd)
    assert st == 0
    c = ctx_for(wl)
    Jdg = dev(Jd)
    Dg = host(c.isc_bilu0(Jdg))
    sc = np.abs(Dinv_o * COL[None, None, :] / COL[None, :, None]).max(axis=(1, 2))
    err = np.abs((Dg - Dinv_o) * COL[None, None, :] / COL[None, :, None]).max(axis=(1, 2))
    assert np.all(err <= 1e-10 * sc)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((m.n, 8)) * COL[None, :]
    y_o = m.spmv(Jd, x)
    y_g = host(c.isc_spmv(Jdg, dev(x)))
    assert np.all(np.abs(y_g - y_o).max(axis=0) <= 1e-12 * np.abs(y_o).max(axis=0))
    z_o = m.bilu0_apply(LU, Dinv_o, x)
    z_g = host(c.isc_bilu0_apply(Jdg, dev(Dinv_o.reshape(m.n, 8, 8)), dev(x)))
    assert np.all(np.abs(z_g - z_o).max(axis=0) <= 1e-10 * np.abs(z_o).max(axis=0))
    # the GMRES iteration's w = A M^-1 x in one pass
    w_o = m.spmv(Jd, z_o)
    z_f, w_f = c.isc_bilu0_apply_spmv(Jdg, dev(Dinv_o.reshape(m.n, 8, 8)), dev(x))
    z_f, w_f = host(z_f), host(w_f)
    assert np.all(np.abs(z_f - z_o).max(axis=0) <= 1e-10 * np.abs(z_o).max(axis=0))
    assert np.all(np.abs(w_f - w_o).max(axis=0) <= 1e-10 * np.abs(w_o).max(axis=0))


@pytest.mark.parametrize("name,seed", [("tiny:13x7x5", 61), ("C1", 62), ("tiny:9x17x6", 63)])
def test_sync_free_factor_equals_level_factor_bitwise(name, seed, monkeypatch):
    """The factor as one cooperative launch (each row awaits its lower
    neighbours' D^-1 as they are published) and as one launch per hyperplane
    run the same per-row arithmetic, so D^-1 agrees bit for bit, and so do
    the applies built on it."""
    wl, m, u, F, J = _decoupled_case(name, seed)
    st, Jd, Fd, _ = m.decouple(J, F)
    c_sf = ctx_for(wl)
    monkeypatch.setenv("ISC_LEVEL_SWEEPS", "1")
    c_lv = ctx_for(wl)
    Jdg = dev(Jd)
    D_sf = c_sf.isc_bilu0(Jdg)
    D_lv = c_lv.isc_bilu0(Jdg)
    torch.cuda.synchronize()
    assert torch.equal(D_sf, D_lv)
    x = dev(np.random.default_rng(seed).standard_normal((m.n, 8)) * COL[None, :])
    assert torch.equal(c_sf.isc_bilu0_apply(Jdg, D_sf, x), c_lv.isc_bilu0_apply(Jdg, D_lv, x))


@pytest.mark.parametrize("level", ["0", "1"])
def test_factor_reports_singular_pivot_without_hanging(level, monkeypatch):
    """A column of three cells whose off-diagonal blocks are the identity:
    D_0 = I, D_1 = I - I I = 0 is singular.  Both factor schedules report
    cell 1; in the sync-free one the singular row still publishes a block, so
    the row after it finishes instead of waiting."""
    from paper_1811_11992_amd import isc
    wl = I.make_workload("tiny:1x1x3")
    m = O.Model(wl)
    Jd = np.zeros((m.row_ptr[-1], 8, 8))
    Jd[:] = np.eye(8)
    monkeypatch.setenv("ISC_LEVEL_SWEEPS", level)
    c = ctx_for(wl)
    with pytest.raises(isc.IscError, match="singular pivot block at cell 1"):
        c.isc_bilu0(dev(Jd))
    st, LU, Dinv_o = m.bilu0(Jd)
    assert st == -4


@pytest.mark.parametrize("coop,bpw", [("1", "1"), ("0", "1"), ("0", "2")])
@pytest.mark.parametrize("name,seed", [("tiny:1x1x6", 40), ("tiny:13x7x5", 41), ("C1", 42)])
def test_sync_free_sweeps_equal_level_sweeps_bitwise(name, seed, coop, bpw, monkeypatch):
    """The single-launch triangular sweeps (rows wait for their predecessors'
    published values) and the one-launch-per-level sweeps do the same
    arithmetic in the same order, so their results agree bit for bit; several
    applications in a row check that each sweep leaves its private buffer
    ready for the next.  The backward sweep fused with the SpMV gives the same
    z; its w = A z adds the lower blocks' products to the upper ones the sweep
    already formed, so it agrees with the separate SpMV to rounding (and bit
    for bit under level sweeps, which run the separate SpMV).  Each schedule
    is checked: the cooperative static one (the default), and tickets with one
    brick or with two independent bricks per workgroup."""
    wl, m, u, F, J = _decoupled_case(name, seed)
    st, Jd, Fd, _ = m.decouple(J, F)
    monkeypatch.setenv("ISC_SWEEP_COOP", coop)
    monkeypatch.setenv("ISC_BRICKS_PER_WG", bpw)
    c_sf = ctx_for(wl)
    monkeypatch.setenv("ISC_LEVEL_SWEEPS", "1")
    c_lv = ctx_for(wl)
    Jdg = dev(Jd)
    D = c_sf.isc_bilu0(Jdg)
    rng = np.random.default_rng(seed)
    for rep in range(4):
        x = dev(rng.standard_normal((m.n, 8)) * COL[None, :])
        z_sf = c_sf.isc_bilu0_apply(Jdg, D, x)
        z_lv = c_lv.isc_bilu0_apply(Jdg, D, x)
        torch.cuda.synchronize()
        assert torch.equal(z_sf, z_lv), rep
        # backward sweep fused with the SpMV: the same z, and w equal to the separate SpMV
        w_ref = c_sf.isc_spmv(Jdg, z_sf)
        # rounding bound of a sum of products, elementwise: |z_i| + sum |A_ij| |z_j|
        bound = c_sf.isc_spmv(Jdg.abs(), z_sf.abs())
        for c in (c_sf, c_lv):
            z_f, w_f = c.isc_bilu0_apply_spmv(Jdg, D, x)
            torch.cuda.synchronize()
            assert torch.equal(z_f, z_sf), rep
            assert bool(((w_f - w_ref).abs() <= 1e-13 * bound).all()), rep
        assert torch.equal(c_lv.isc_bilu0_apply_spmv(Jdg, D, x)[1], w_ref)


@pytest.mark.parametrize("coop", ["1", "0"])
def test_sweep_wait_limit_ends_in_an_error_not_a_hang(coop, monkeypatch):
    """The sync-free sweeps bound every wait in wall-clock time.  With the
    limit forced down from the host to one tick, rows that have to wait for
    their predecessors give up, every wavefront still exits, and the apply
    reports the timeout as an error; a context with the normal limit applies
    the same factor without error."""
    from paper_1811_11992_amd import isc
    wl = I.make_workload("tiny:60x60x20")
    monkeypatch.setenv("ISC_SWEEP_COOP", coop)
    monkeypatch.setenv("ISC_SWEEP_WAIT_TICKS", "1")
    c_tiny = ctx_for(wl)
    monkeypatch.delenv("ISC_SWEEP_WAIT_TICKS")
    c_ok = ctx_for(wl)
    u0 = dev(wl.u0)
    F, J = c_ok.isc_assemble(u0, u0, wl.dt)
    c_ok.isc_decouple(J, F)
    D = c_ok.isc_bilu0(J)
    r = torch.randn((wl.ncell, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(isc.IscError, match="waited too long"):
        c_tiny.isc_bilu0_apply(J, D, r)
    z = c_ok.isc_bilu0_apply(J, D, r)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(z).all())


@pytest.mark.parametrize("name,seed", [("tiny:13x7x5", 21), ("C1", 22)])
def test_solve_reaches_tolerance_and_matches_tight_oracle_solution(name, seed):
    from paper_1811_11992_amd import isc
    wl, m, u, F, J = _decoupled_case(name, seed)
    st, Jd, Fd, _ = m.decouple(J, F)
    b = -Fd
    c = ctx_for(wl)
    x, info, st = c.isc_solve(dev(Jd), dev(b), isc.solve_opts(rtol=1e-8))
    assert st == 0 and info.relres_true <= 1e-8
    xg = host(x)
    r = b - m.spmv(Jd, xg)
    assert np.linalg.norm(r) <= 1.01e-8 * np.linalg.norm(b)
    st, x_ref, inf = m.gmres(Jd, b, rtol=1e-13, max_restarts=60)
    assert st == 0
    err = np.abs((xg - x_ref) / COL).max(axis=0)
    ref = np.abs(x_ref / COL).max(axis=0) + 1e-300
    assert np.all(err <= 1e-5 * ref.max()), err / ref.max()


@pytest.mark.parametrize("name,seed,restart,coop,bpw,fold", [("tiny:13x7x5", 23, 30, "1", "1", "1"),
                                                             ("C1", 24, 30, "0", "2", "1"),
                                                             ("C1", 25, 10, "1", "1", "1"),
                                                             ("C1", 26, 10, "1", "1", "0")])
def test_solve_with_update_in_the_sweep_matches_separate_update(name, seed, restart, coop, bpw, fold, monkeypatch):
    """With sync-free sweeps the FP64 GMRES can do each iteration's delayed
    Gram-Schmidt update inside the next iteration's forward sweep
    (ISC_FOLD_UPDATE=1); by default, and with level sweeps, it runs as a pass
    of its own.  The per-element arithmetic is the
    same, so both reach the tolerance after the same number of iterations and
    give the same solution to rounding, also across many restarts (GMRES(10)
    needs about 25 cycles on the C1 case, as does the oracle's GMRES)."""
    from paper_1811_11992_amd import isc
    wl, m, u, F, J = _decoupled_case(name, seed)
    st, Jd, Fd, _ = m.decouple(J, F)
    b = dev(-Fd)
    monkeypatch.setenv("ISC_SWEEP_COOP", coop)
    monkeypatch.setenv("ISC_BRICKS_PER_WG", bpw)
    monkeypatch.setenv("ISC_FOLD_UPDATE", fold)
    c_sf = ctx_for(wl)
    monkeypatch.setenv("ISC_LEVEL_SWEEPS", "1")
    c_lv = ctx_for(wl)
    o = isc.solve_opts(rtol=1e-9, restart=restart, max_restarts=200)
    x_sf, inf_sf, st_sf = c_sf.isc_solve(dev(Jd), b, o)
    x_lv, inf_lv, st_lv = c_lv.isc_solve(dev(Jd), b, o)
    assert st_sf == 0 and st_lv == 0
    assert inf_sf.relres_true <= 1e-9 and inf_lv.relres_true <= 1e-9
    # rounding differences may move the stopping iteration of a long run a little
    assert abs(inf_sf.iters - inf_lv.iters) <= max(1, inf_lv.iters // 50), (inf_sf.iters, inf_lv.iters)
    xs, xl = host(x_sf), host(x_lv)
    err = np.abs((xs - xl) / COL).max(axis=0)
    ref = np.abs(xl / COL).max(axis=0).max() + 1e-300
    assert np.all(err <= 1e-6 * ref), err / ref


def test_newton_root_matches_oracle_on_c1_first_step():
    wl = I.make_workload("C1")
    m = O.Model(wl)
    c = ctx_for(wl)
    tol = 1e-11
    uo = wl.u0.copy()
    u_or = uo.copy()
    for _ in range(20):
        st, u_or, info = m.newton_step(u_or, uo, wl.dt, tol=tol)
        assert st == 0
        if info.converged:
            break
    assert info.converged
    ug = dev(uo)
    ugo = dev(uo)
    for _ in range(20):
        st, inf = c.isc_newton_step(ug, ugo, wl.dt, tol=tol)
        assert st == 0, st
        if inf.converged:
            break
    assert inf.converged
    u_g = host(ug)
    rel = np.abs(u_g - u_or).max(axis=1) / np.maximum(np.abs(u_or).max(axis=1), FLOOR)
    assert np.all(rel <= 1e-9), rel
    F = m.residual(u_g, uo, wl.dt)
    assert m.scaled_norm(F, wl.dt) <= 1e-10


def _drive(step_fn, copy, u0, dt, nsteps, max_newton=12):
    """Time loop used for both sides in parity mode: Newton to tol 1e-10, then
    one extra iteration (tol 0 forces a solve) so that both sit at the root to
    rounding; a failed step is retried with half the step (at most 4 times)."""
    u = copy(u0)
    hist, dts = [copy(u)], []
    for _ in range(nsteps):
        uo = copy(u)
        dt_s = dt
        for cut in range(5):
            ok = False
            for _k in range(max_newton + 1):
                st, conv = step_fn(u, uo, dt_s, 1e-10)
                if st != 0:
                    break
                if conv:
                    ok = True
                    break
            if ok:
                st, _ = step_fn(u, uo, dt_s, 0.0)
                assert st == 0
                break
            u = copy(uo)
            dt_s *= 0.5
        assert ok
        hist.append(copy(u))
        dts.append(dt_s)
    return hist, dts


def test_run_c1_matches_oracle_per_step():
    wl = I.make_workload("C1")
    m = O.Model(wl)

    def o_step(u, uo, dt, tol):
        st, v, info = m.newton_step(u, uo, dt, tol=tol)
        u[...] = v
        return st, bool(info.converged)

    hist_o, dts_o = _drive(o_step, lambda a: np.array(a, copy=True), wl.u0, wl.dt, wl.nsteps)
    c = ctx_for(wl)

    def g_step(u, uo, dt, tol):
        st, info = c.isc_newton_step(u, uo, dt, tol=tol)
        return st, bool(info.converged)

    hist_g, dts_g = _drive(g_step, lambda a: dev(a) if isinstance(a, np.ndarray) else a.clone(), wl.u0,
                           wl.dt, wl.nsteps)
    assert dts_g == dts_o
    for s in range(wl.nsteps):
        ug = host(hist_g[s + 1])
        rel = np.abs(ug - hist_o[s + 1]).max(axis=1) / np.maximum(np.abs(hist_o[s + 1]).max(axis=1), FLOOR)
        assert np.all(rel <= 1e-9), (s, rel)
        F = m.residual(ug, host(hist_g[s]), dts_g[s])
        assert m.scaled_norm(F, dts_g[s]) <= 1e-10


def _dense(m, Jd):
    """The decoupled matrix as a dense array (unit diagonal blocks)."""
    n = m.n
    A = np.zeros((8 * n, 8 * n))
    for i in range(n):
        for b in range(m.row_ptr[i], m.row_ptr[i + 1]):
            k = m.col_idx[b]
            A[8 * i:8 * i + 8, 8 * k:8 * k + 8] = np.eye(8) if k == i else Jd[b]
    return A


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["identity", "chain", "zero_rhs"])
def test_solve_with_exact_preconditioner_and_zero_rhs(case, precision):
    """Breakdown paths of the Krylov step.  With no off-diagonal blocks
    (A = I) and on a one-cell-wide chain, BILU(0) is exact (M = A), so the
    second basis vector is zero: omega = 0 flags the breakdown and the
    one-column solution is already exact.  A zero right-hand side returns
    x = 0 at once.  Checked against a dense solve."""
    from paper_1811_11992_amd import isc
    name = "tiny:9x1x1" if case == "chain" else "tiny:4x3x2"
    wl, m, u, F, J = _decoupled_case(name, 41)
    st, Jd, Fd, _ = m.decouple(J, F)
    assert st == 0
    Jd = Jd.copy()
    for i in range(m.n):
        for b in range(m.row_ptr[i], m.row_ptr[i + 1]):
            if m.col_idx[b] == i:
                Jd[b] = np.eye(8)
            elif case == "identity":
                Jd[b] = 0.0
    b = np.zeros_like(Fd) if case == "zero_rhs" else -Fd
    kw = dict(rtol=1e-8)
    if precision == "mixed":
        c = ctx_for(wl, inner_iters=6)
        kw.update(precision=isc.ISC_MIXED, inner_iters=6)
    else:
        c = ctx_for(wl)
    x, info, st = c.isc_solve(dev(Jd), dev(b), isc.solve_opts(**kw))
    assert st == 0
    xg = host(x)
    if case == "zero_rhs":
        assert info.iters == 0 and np.array_equal(xg, np.zeros_like(xg))
        return
    x_ref = np.linalg.solve(_dense(m, Jd), b.reshape(-1)).reshape(m.n, 8)
    err = np.abs((xg - x_ref) / COL).max() / np.abs(x_ref / COL).max()
    if precision == "fp64":   # one column is the exact solution, up to rounding
        assert info.iters <= 2, info.iters
        assert info.relres_true <= 1e-10 and err <= 1e-9, (info.relres_true, err)
    else:                     # FP32 inner solves: each outer column gains about 7 digits
        assert info.relres_true <= 1e-8 and err <= 1e-6, (info.relres_true, err)


# ------------------------------------------------------------ precision form
@pytest.mark.parametrize("level", ["0", "1"])
@pytest.mark.parametrize("name,seed", [("tiny:13x7x5", 31), ("C1", 32)])
def test_mixed_solve_reaches_fp64_tolerance(name, seed, level, monkeypatch):
    """FP32 BILU(0) + FP32 inner GMRES inside FP64 FGMRES(30): the FP64 true
    residual still meets 1e-8 and the solution matches a tight FP64 solve.
    Under both schedules: the sync-free factor rounds the FP64 blocks as it
    loads them, the per-hyperplane one factors an FP32 copy of the matrix."""
    from paper_1811_11992_amd import isc
    monkeypatch.setenv("ISC_LEVEL_SWEEPS", level)
    wl, m, u, F, J = _decoupled_case(name, seed)
    st, Jd, Fd, _ = m.decouple(J, F)
    b = -Fd
    c = ctx_for(wl, inner_iters=6)
    x, info, st = c.isc_solve(dev(Jd), dev(b), isc.solve_opts(rtol=1e-8, precision=isc.ISC_MIXED, inner_iters=6))
    assert st == 0 and info.relres_true <= 1e-8
    # one inner solve per column, plus at most one per cycle whose residual test ended the cycle
    assert info.inner_iters_total % 6 == 0
    assert 6 * info.iters <= info.inner_iters_total <= 6 * (info.iters + info.restarts + 1)
    xg = host(x)
    assert np.linalg.norm(b - m.spmv(Jd, xg)) <= 1.01e-8 * np.linalg.norm(b)
    st, x_ref, _ = m.gmres(Jd, b, rtol=1e-13, max_restarts=60)
    err = np.abs((xg - x_ref) / COL).max(axis=0)
    assert np.all(err <= 1e-5 * np.abs(x_ref / COL).max()), err


def test_mixed_newton_root_matches_fp64_oracle():
    from paper_1811_11992_amd import isc
    wl = I.make_workload("C1")
    m = O.Model(wl)
    c = ctx_for(wl, inner_iters=6)
    lin = isc.solve_opts(precision=isc.ISC_MIXED, inner_iters=6)

    def o_step(u, uo, dt, tol):
        st, v, info = m.newton_step(u, uo, dt, tol=tol)
        u[...] = v
        return st, bool(info.converged)

    def g_step(u, uo, dt, tol):
        st, info = c.isc_newton_step(u, uo, dt, tol=tol, lin=lin)
        return st, bool(info.converged)

    hist_o, dts_o = _drive(o_step, lambda a: np.array(a, copy=True), wl.u0, wl.dt, 3)
    hist_g, dts_g = _drive(g_step, lambda a: dev(a) if isinstance(a, np.ndarray) else a.clone(), wl.u0, wl.dt, 3)
    assert dts_g == dts_o
    for s in range(3):
        ug = host(hist_g[s + 1])
        rel = np.abs(ug - hist_o[s + 1]).max(axis=1) / np.maximum(np.abs(hist_o[s + 1]).max(axis=1), FLOOR)
        assert np.all(rel <= 1e-8), (s, rel)
        assert m.scaled_norm(m.residual(ug, host(hist_g[s]), dts_g[s]), dts_g[s]) <= 1e-10
