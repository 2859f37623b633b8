"""Pins of the oracle's CPR preconditioner (CPU only).

Each part is checked against something other than the oracle's own code:
the definition of the pressure matrix and of the Galerkin product written
densely with numpy, the block form of one red-black Gauss-Seidel sweep, the
two-level V-cycle written out densely, the minimal-residual property of the
GMRES pressure solve over an explicitly built Krylov space, the two-stage
formula with an exact pressure solve, exactness on a one-cell-wide chain, a
dense direct solve, and the contraction of the multigrid cycle."""
import numpy as np
import pytest

import oracle as O
from paper_1811_11992_amd import inputs as I


def _system(name, seed=None):
    wl = I.make_workload(name)
    m = O.Model(wl)
    u = wl.u0 if seed is None else I.random_states(wl, seed=seed)
    F, J = m.assemble(u, wl.u0, wl.dt)
    st, Jd, Fd, bad = m.decouple(J, F)
    assert st == 0
    return wl, m, Jd, -Fd


def _dense_blocks(m, Jd):
    n = m.n
    A = np.zeros((8 * n, 8 * n))
    for i in range(n):
        for b in range(m.row_ptr[i], m.row_ptr[i + 1]):
            j = m.col_idx[b]
            A[8 * i:8 * i + 8, 8 * j:8 * j + 8] = Jd[b]
    return A


def _pressure_dense(m, Jd):
    n = m.n
    Ap = np.zeros((n, n))
    for i in range(n):
        for b in range(m.row_ptr[i], m.row_ptr[i + 1]):
            Ap[i, m.col_idx[b]] = Jd[b, 0, 0]
    return Ap


def _aggregation(dims):
    """Piecewise-constant prolongation of 2x2x2 boxes, from its definition."""
    nx, ny, nz = dims
    cx, cy, cz = (nx + 1) // 2, (ny + 1) // 2, (nz + 1) // 2
    P = np.zeros((nx * ny * nz, cx * cy * cz))
    for iz in range(nz):
        for iy in range(ny):
            for ix in range(nx):
                P[ix + nx * (iy + ny * iz), ix // 2 + cx * (iy // 2 + cy * (iz // 2))] = 1.0
    return P, (cx, cy, cz)


def _colours(dims):
    nx, ny, nz = dims
    i = np.arange(nx * ny * nz)
    return (i % nx + (i // nx) % ny + i // (nx * ny)) % 2


def _rbgs_dense(A, b, x, col, first):
    """One red-black sweep in block form: each colour's unknowns solve their
    own rows with the other colour's current values (same-colour couplings
    are absent on the 7-point stencil, so the colour block is diagonal)."""
    x = x.copy()
    for c in (first, 1 - first):
        S = col == c
        T = ~S
        Ass = A[np.ix_(S, S)]
        assert np.count_nonzero(Ass - np.diag(np.diag(Ass))) == 0
        x[S] = (b[S] - A[np.ix_(S, T)] @ x[T]) / np.diag(Ass)
    return x


def test_pressure_matrix_and_galerkin_levels():
    wl, m, Jd, b = _system("tiny:13x7x5", seed=5)
    c = O.CPR(m, Jd)
    assert c.nlevels == 3
    A = _pressure_dense(m, Jd)
    assert np.array_equal(c.level_dense(0), A)
    assert np.allclose(np.diag(A), 1.0)        # the decoupled diagonal blocks are the identity
    dims = (wl.nx, wl.ny, wl.nz)
    for l in range(1, c.nlevels):
        P, cdims = _aggregation(dims)
        Ac = P.T @ A @ P
        got = c.level_dense(l)
        assert c.level_dims(l)[0] == cdims
        assert np.abs(got - Ac).max() <= 1e-13 * np.abs(Ac).max()
        # still a 7-point stencil on the coarse grid
        cnx, cny, cnz = cdims
        for I_, row in enumerate(got):
            for J_ in np.nonzero(row)[0]:
                d = abs(J_ - I_)
                assert d in (0, 1, cnx, cnx * cny)
        A, dims = Ac, cdims
    assert np.prod(dims) <= O.CPR_COARSEST


@pytest.mark.parametrize("first", [0, 1])
def test_red_black_sweep_matches_block_form(first):
    wl, m, Jd, _ = _system("tiny:13x7x5", seed=6)
    c = O.CPR(m, Jd)
    rng = np.random.default_rng(11)
    for l in range(c.nlevels - 1):
        (dims, n) = c.level_dims(l)
        A = c.level_dense(l)
        b = rng.standard_normal(n)
        x0 = rng.standard_normal(n)
        got = c.smooth(l, b, x0, first)
        want = _rbgs_dense(A, b, x0, _colours(dims), first)
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_two_level_vcycle_matches_its_dense_form():
    wl, m, Jd, _ = _system("tiny:8x6x2", seed=7)
    c = O.CPR(m, Jd, nu=2, cf=1.5)
    assert c.nlevels == 2
    A = c.level_dense(0)
    dims, n = c.level_dims(0)
    col = _colours(dims)
    P, _ = _aggregation(dims)
    Ac = P.T @ A @ P
    rng = np.random.default_rng(3)
    b = rng.standard_normal(n)
    x = np.zeros(n)
    for _ in range(2):
        x = _rbgs_dense(A, b, x, col, 0)
    x = x + 1.5 * P @ np.linalg.solve(Ac, P.T @ (b - A @ x))
    for _ in range(2):
        x = _rbgs_dense(A, b, x, col, 1)
    got = c.vcycle(b)
    assert np.abs(got - x).max() <= 1e-11 * np.abs(x).max()


@pytest.mark.parametrize("k", [1, 3, 5])
def test_pressure_solve_minimises_the_residual_over_its_krylov_space(k):
    # the pressure matrix of a physical state (at the initial state the
    # decoupled pressure rows are diagonally dominant M-matrix rows)
    wl, m, Jd, _ = _system("tiny:13x7x5")
    c = O.CPR(m, Jd, p_iters=k)
    A = c.level_dense(0)
    n = A.shape[0]
    # the V-cycle is a fixed linear map: its matrix, column by column
    M = np.column_stack([c.vcycle(e) for e in np.eye(n)])
    rng = np.random.default_rng(k)
    r = rng.standard_normal(n)
    # orthonormal basis of the Krylov space span{r, (AM) r, ..., (AM)^(k-1) r},
    # each new direction orthogonalised by a Householder QR of the whole set
    Q = (r / np.linalg.norm(r))[:, None]
    for _ in range(k - 1):
        Q, _ = np.linalg.qr(np.column_stack([Q, A @ M @ Q[:, -1]]))
    coef, *_ = np.linalg.lstsq(A @ M @ Q, r, rcond=None)
    want = M @ (Q @ coef)
    got = c.pressure(r)
    # both minimise ||r - A x|| over the same space
    res_got, res_want = np.linalg.norm(r - A @ got), np.linalg.norm(r - A @ want)
    assert abs(res_got - res_want) <= 1e-10 * np.linalg.norm(r)
    assert np.abs(got - want).max() <= 1e-8 * np.abs(want).max()
    # and the residual falls with every step at this state
    assert res_got < 0.2 ** k * np.linalg.norm(r)


def test_cpr_apply_is_the_two_stage_formula():
    wl, m, Jd, _ = _system("tiny:4x3x2", seed=9)     # 24 cells: the pressure solve is direct
    c = O.CPR(m, Jd)
    assert c.nlevels == 1
    A = _dense_blocks(m, Jd)
    Ap = _pressure_dense(m, Jd)
    st, LU, Dinv = m.bilu0(Jd)
    rng = np.random.default_rng(4)
    r = rng.standard_normal((m.n, 8))
    z1 = np.zeros((m.n, 8))
    z1[:, 0] = np.linalg.solve(Ap, r[:, 0])
    r2 = r.ravel() - A @ z1.ravel()
    want = z1 + m.bilu0_apply(LU, Dinv, r2.reshape(m.n, 8))
    got = c.apply(r)
    assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()
    # with multigrid levels the same split holds for the oracle's own pressure stage
    wl, m, Jd, _ = _system("tiny:13x7x5", seed=9)
    c = O.CPR(m, Jd)
    A = _dense_blocks(m, Jd)
    st, LU, Dinv = m.bilu0(Jd)
    r = rng.standard_normal((m.n, 8))
    z1 = np.zeros((m.n, 8))
    z1[:, 0] = c.pressure(r[:, 0])
    want = z1 + m.bilu0_apply(LU, Dinv, (r.ravel() - A @ z1.ravel()).reshape(m.n, 8))
    got = c.apply(r)
    assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()


def test_fgmres_cpr_is_exact_on_a_chain():
    # a one-cell-wide chain: block ILU(0) is the exact block LU, so CPR is exact
    wl, m, Jd, b = _system("tiny:12x1x1", seed=10)
    st, x, info = m.fgmres_cpr(Jd, b, rtol=1e-14)
    assert st == 0 and info.iters == 1 and info.relres_true <= 1e-13


@pytest.mark.parametrize("name", ["tiny:4x3x2", "tiny:13x7x5"])
def test_fgmres_cpr_matches_a_dense_solve(name):
    wl, m, Jd, b = _system(name, seed=12)
    st, x, info = m.fgmres_cpr(Jd, b, rtol=1e-12)
    assert st == 0 and info.relres_true <= 1e-12
    xd = np.linalg.solve(_dense_blocks(m, Jd), b.ravel()).reshape(m.n, 8)
    scale = np.abs(xd).max(axis=0) + 1e-300
    assert np.all(np.abs(x - xd).max(axis=0) <= 1e-8 * scale)


def test_multigrid_cycle_contracts_and_cpr_beats_bilu0_on_c1():
    wl, m, Jd, b = _system("C1")
    c = O.CPR(m, Jd)
    assert c.nlevels >= 2
    # with an unscaled coarse correction the V-cycle is a convergent stationary
    # iteration on the pressure matrix (about 0.5 per cycle here)
    c1 = O.CPR(m, Jd, nu=2, cf=1.0)
    A = c1.level_dense(0)
    rng = np.random.default_rng(2)
    rhs = rng.standard_normal(m.n)
    x = np.zeros(m.n)
    r0 = np.linalg.norm(rhs)
    for _ in range(8):
        x = x + c1.vcycle(rhs - A @ x)
    assert np.linalg.norm(rhs - A @ x) <= 0.6 ** 8 * r0
    st, _, info_cpr = m.fgmres_cpr(Jd, b, rtol=1e-8)
    st2, _, info_ilu = m.gmres(Jd, b, rtol=1e-8)
    assert st == 0 and st2 == 0
    assert info_cpr.iters < info_ilu.iters
