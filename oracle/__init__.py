"""Python access to the CPU oracle (test infrastructure only).

The oracle is a plain, serial FP64 CPU implementation of the simulator's
Newton hot path written from the paper.  It checks the GPU library and is
never called by it.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this module.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from paper_1811_11992_amd import inputs as I

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("relres_est", ctypes.c_double), ("relres_true", ctypes.c_double)]


class NewtonInfo(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int32), ("iters_lin", ctypes.c_int32),
                ("status", ctypes.c_int32), ("res_scaled", ctypes.c_double),
                ("relres_true", ctypes.c_double)]


class StepInfo(ctypes.Structure):
    _fields_ = [("newton_its", ctypes.c_int32), ("lin_its", ctypes.c_int32),
                ("cuts", ctypes.c_int32), ("dt_used", ctypes.c_double),
                ("res_final", ctypes.c_double)]


CPR_P_ITERS, CPR_NU, CPR_CF = 6, 2, 1.5   # defaults of the CPR preconditioner
CPR_COARSEST = 64

DIAG = dict(So=0, xHO=1, y0=2, Z=8, rho_w=9, rho_o=10, rho_g=11, mu_w=12, mu_o=13, mu_g=14,
            phi=15, phif=16, krw=17, kro=18, krg=19, Hw=20, Ho=21, Hg=22, KT=23, r0=24,
            acc0=28, K_W=36, K_LO=37, K_HO=38, Hv_W=39, Hg_O2=40)
NDIAG = 41


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b  # noqa: F401  (oracle/build.py)
            _b.build()
        L = ctypes.CDLL(path)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p, _dp, ctypes.c_double, _dp,
                                 ctypes.c_void_p, ctypes.c_int32]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_ncell.argtypes = [ctypes.c_void_p]
        L.orc_nnzb.argtypes = [ctypes.c_void_p]
        L.orc_nnzb.restype = ctypes.c_int32
        L.orc_pattern.argtypes = [ctypes.c_void_p, _ip, _ip]
        L.orc_set_params.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_set_heater.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double]
        L.orc_perf_info.argtypes = [ctypes.c_void_p, _ip, _ip, _dp, _dp]
        L.orc_diag.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_zfactor.restype = ctypes.c_double
        L.orc_zfactor.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp]
        L.orc_gas_viscosity.restype = ctypes.c_double
        L.orc_gas_viscosity.argtypes = [ctypes.c_void_p, ctypes.c_double, _dp]
        L.orc_residual.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, _dp]
        L.orc_assemble.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, _dp, _dp]
        L.orc_sources.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.orc_decouple.argtypes = [ctypes.c_void_p, _dp, _dp, _ip]
        L.orc_bilu0.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.orc_bilu0_apply.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp]
        L.orc_spmv.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.orc_gmres.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_double, ctypes.POINTER(SolveInfo)]
        L.orc_bicgstab.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, ctypes.c_int32, ctypes.c_double,
                                   ctypes.POINTER(SolveInfo)]
        L.orc_scaled_norm.restype = ctypes.c_double
        L.orc_scaled_norm.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double]
        L.orc_update.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_newton_step.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                      ctypes.POINTER(NewtonInfo)]
        L.orc_run.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                              ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                              ctypes.POINTER(StepInfo), _dp]
        L.orc_cpr_create.restype = ctypes.c_void_p
        L.orc_cpr_create.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double]
        L.orc_cpr_destroy.argtypes = [ctypes.c_void_p]
        L.orc_cpr_nlevels.argtypes = [ctypes.c_void_p]
        L.orc_cpr_level_dims.argtypes = [ctypes.c_void_p, ctypes.c_int32, _ip]
        L.orc_cpr_level_dense.argtypes = [ctypes.c_void_p, ctypes.c_int32, _dp]
        L.orc_cpr_smooth.argtypes = [ctypes.c_void_p, ctypes.c_int32, _dp, _dp, ctypes.c_int32]
        L.orc_cpr_vcycle.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_cpr_pressure.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_cpr_apply.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_fgmres_cpr.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(SolveInfo)]
        L.orc_ncwell.restype = ctypes.c_int32
        L.orc_ncwell.argtypes = [ctypes.c_void_p]
        L.orc_well_state.argtypes = [ctypes.c_void_p, _dp, _ip]
        L.orc_set_well_state.argtypes = [ctypes.c_void_p, _dp, _ip]
        L.orc_well_controls.restype = ctypes.c_int32
        L.orc_well_controls.argtypes = [ctypes.c_void_p, _dp]
        L.orc_well_solve.restype = ctypes.c_int32
        L.orc_well_solve.argtypes = [ctypes.c_void_p, _dp]
        L.orc_well_border.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp]
        L.orc_well_scaled_norm.restype = ctypes.c_double
        L.orc_well_scaled_norm.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double]
        if hasattr(L, "orc_adjoint_step"):
            L.orc_oil_rate.restype = ctypes.c_double
            L.orc_oil_rate.argtypes = [ctypes.c_void_p, _dp]
            L.orc_adjoint_step.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, _dp, _dp,
                                           ctypes.c_double, _dp, _dp, _dp]
        _LIB = L
    return _LIB


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous, (a.dtype, a.flags)
    return a.ctypes.data_as(_dp)


def _ip_(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_ip)


class Model:
    """One oracle model (grid + physics card + rock + wells)."""

    def __init__(self, wl: I.Workload, fluid: I.Fluid | None = None):
        L = lib()
        self.wl = wl
        self.fluid = fluid if fluid is not None else I.physics_card()
        self._grid = wl.grid()
        self._wells, self._keep = wl.well_structs()
        self.logk = np.ascontiguousarray(wl.logk, dtype=np.float64)
        self.poro = np.ascontiguousarray(wl.poro, dtype=np.float64)
        self.h = L.orc_create(ctypes.byref(self._grid), ctypes.byref(self.fluid), _p(self.logk),
                              wl.kv_over_kh, _p(self.poro), ctypes.cast(self._wells, ctypes.c_void_p),
                              len(wl.wells))
        self.n = wl.ncell
        self.nnzb = L.orc_nnzb(self.h)
        self.row_ptr = np.zeros(self.n + 1, np.int32)
        self.col_idx = np.zeros(self.nnzb, np.int32)
        L.orc_pattern(self.h, _ip_(self.row_ptr), _ip_(self.col_idx))

    def __del__(self):
        # at interpreter shutdown the module globals may already be gone
        if getattr(self, "h", None) and _LIB is not None and callable(lib):
            _LIB.orc_destroy(self.h)
            self.h = None

    # ---- setup
    def set_params(self, logk=None, A=None):
        lk = None if logk is None else np.ascontiguousarray(logk, np.float64)
        a = None if A is None else np.ascontiguousarray(A, np.float64)
        lib().orc_set_params(self.h, _p(lk), _p(a))

    def set_heater(self, cell, rate_W):
        lib().orc_set_heater(self.h, int(cell), float(rate_W))

    def perf_info(self):
        npf = sum(len(w["cells"]) for w in self.wl.wells)
        cells = np.zeros(npf, np.int32)
        kinds = np.zeros(npf, np.int32)
        wi = np.zeros(npf)
        q = np.zeros(npf)
        lib().orc_perf_info(self.h, _ip_(cells), _ip_(kinds), _p(wi), _p(q))
        return cells, kinds, wi, q

    # ---- controlled wells (kinds 3, 4)
    @property
    def ncwell(self):
        return lib().orc_ncwell(self.h)

    @property
    def ncperf(self):
        return sum(len(w["cells"]) for w in self.wl.wells if w["kind"] in (I.WELL_PRODUCER, I.WELL_INJECTOR))

    def well_state(self):
        bhp = np.zeros(max(1, self.ncwell))
        on = np.zeros(max(1, self.ncwell), np.int32)
        lib().orc_well_state(self.h, _p(bhp), _ip_(on))
        return bhp[:self.ncwell].copy(), on[:self.ncwell].copy()

    def set_well_state(self, bhp, on_limit):
        b = np.ascontiguousarray(np.resize(np.asarray(bhp, np.float64), max(1, self.ncwell)))
        o = np.ascontiguousarray(np.resize(np.asarray(on_limit, np.int32), max(1, self.ncwell)))
        lib().orc_set_well_state(self.h, _p(b), _ip_(o))

    def well_controls(self, u):
        return lib().orc_well_controls(self.h, _p(np.ascontiguousarray(u, np.float64)))

    def well_solve(self, u):
        return lib().orc_well_solve(self.h, _p(np.ascontiguousarray(u, np.float64)))

    def well_border(self, u):
        """(R[ncw], D[ncw], B[ncp][8], C[ncp][8]) at state u and the current well state."""
        nw, npf = max(1, self.ncwell), max(1, self.ncperf)
        R, D = np.zeros(nw), np.zeros(nw)
        B, C = np.zeros((npf, 8)), np.zeros((npf, 8))
        lib().orc_well_border(self.h, _p(np.ascontiguousarray(u, np.float64)), _p(R), _p(D), _p(B), _p(C))
        return R[:self.ncwell], D[:self.ncwell], B[:self.ncperf], C[:self.ncperf]

    def well_scaled_norm(self, R, dt):
        r = np.ascontiguousarray(np.resize(np.asarray(R, np.float64), max(1, self.ncwell)))
        return lib().orc_well_scaled_norm(self.h, _p(r), float(dt))

    # ---- diagnostics
    def diag(self, u):
        u = np.ascontiguousarray(u, np.float64)
        out = np.zeros((self.n, NDIAG))
        lib().orc_diag(self.h, _p(u), _p(out))
        return out

    # ---- hot path
    def residual(self, u, u_old, dt):
        F = np.zeros((self.n, 8))
        lib().orc_residual(self.h, _p(np.ascontiguousarray(u)), _p(np.ascontiguousarray(u_old)), dt, _p(F))
        return F

    def assemble(self, u, u_old, dt):
        F = np.zeros((self.n, 8))
        J = np.zeros((self.nnzb, 8, 8))
        lib().orc_assemble(self.h, _p(np.ascontiguousarray(u)), _p(np.ascontiguousarray(u_old)),
                           dt, _p(F), _p(J))
        return F, J

    def sources(self, u):
        W = np.zeros((self.n, 8))
        R = np.zeros((self.n, 8))
        lib().orc_sources(self.h, _p(np.ascontiguousarray(u)), _p(W), _p(R))
        return W, R

    def decouple(self, J, F):
        J = np.array(J, dtype=np.float64, order="C")
        F = np.array(F, dtype=np.float64, order="C")
        bad = ctypes.c_int32(-1)
        st = lib().orc_decouple(self.h, _p(J), _p(F), ctypes.byref(bad))
        return st, J, F, bad.value

    def bilu0(self, Jdec):
        LU = np.zeros_like(Jdec)
        Dinv = np.zeros((self.n, 8, 8))
        st = lib().orc_bilu0(self.h, _p(np.ascontiguousarray(Jdec)), _p(LU), _p(Dinv))
        return st, LU, Dinv

    def bilu0_apply(self, LU, Dinv, r):
        z = np.zeros((self.n, 8))
        lib().orc_bilu0_apply(self.h, _p(LU), _p(Dinv), _p(np.ascontiguousarray(r, np.float64)), _p(z))
        return z

    def spmv(self, J, x):
        y = np.zeros((self.n, 8))
        lib().orc_spmv(self.h, _p(np.ascontiguousarray(J)), _p(np.ascontiguousarray(x, np.float64)), _p(y))
        return y

    def gmres(self, Jdec, b, restart=30, max_restarts=20, rtol=1e-8):
        x = np.zeros((self.n, 8))
        info = SolveInfo()
        st = lib().orc_gmres(self.h, _p(np.ascontiguousarray(Jdec)), _p(np.ascontiguousarray(b, np.float64)),
                             _p(x), restart, max_restarts, rtol, ctypes.byref(info))
        return st, x, info

    def bicgstab(self, Jdec, b, max_iters=1000, rtol=1e-8):
        x = np.zeros((self.n, 8))
        info = SolveInfo()
        st = lib().orc_bicgstab(self.h, _p(np.ascontiguousarray(Jdec)), _p(np.ascontiguousarray(b, np.float64)),
                                _p(x), max_iters, rtol, ctypes.byref(info))
        return st, x, info

    def fgmres_cpr(self, Jdec, b, restart=30, max_restarts=20, rtol=1e-8, p_iters=CPR_P_ITERS, nu=CPR_NU,
                   cf=CPR_CF):
        x = np.zeros((self.n, 8))
        info = SolveInfo()
        st = lib().orc_fgmres_cpr(self.h, _p(np.ascontiguousarray(Jdec)), _p(np.ascontiguousarray(b, np.float64)),
                                  _p(x), restart, max_restarts, rtol, p_iters, nu, cf, ctypes.byref(info))
        return st, x, info

    def scaled_norm(self, F, dt):
        return lib().orc_scaled_norm(self.h, _p(np.ascontiguousarray(F, np.float64)), dt)

    def update(self, u, du):
        u = np.array(u, dtype=np.float64, order="C")
        st = lib().orc_update(self.h, _p(u), _p(np.ascontiguousarray(du, np.float64)))
        return st, u

    def oil_rate(self, u):
        return lib().orc_oil_rate(self.h, _p(np.ascontiguousarray(u, np.float64)))

    def adjoint_step(self, u_n, u_nm1, dt_n, lam_np1, dt_np1, g_logk, g_A):
        lam = np.zeros((self.n, 8))
        lp = None if lam_np1 is None else np.ascontiguousarray(lam_np1, np.float64)
        st = lib().orc_adjoint_step(self.h, _p(np.ascontiguousarray(u_n)), _p(np.ascontiguousarray(u_nm1)), dt_n,
                                    _p(lp), None, dt_np1, _p(lam), _p(g_logk), _p(g_A))
        return st, lam

    def newton_step(self, u, u_old, dt, tol=1e-10, restart=30, max_restarts=20, rtol=1e-8):
        u = np.array(u, dtype=np.float64, order="C")
        info = NewtonInfo()
        st = lib().orc_newton_step(self.h, _p(u), _p(np.ascontiguousarray(u_old)), dt, tol, restart,
                                   max_restarts, rtol, ctypes.byref(info))
        return st, u, info

    def run(self, u0, dt, nsteps, tol=1e-10, max_newton=12, restart=30, max_restarts=20, rtol=1e-8,
            keep_history=False):
        u = np.array(u0, dtype=np.float64, order="C")
        steps = (StepInfo * nsteps)()
        hist = np.zeros((nsteps + 1, 8, self.n)) if keep_history else None
        st = lib().orc_run(self.h, _p(u), dt, nsteps, tol, max_newton, restart, max_restarts, rtol,
                           steps, _p(hist))
        return st, u, [dict(newton=s.newton_its, lin=s.lin_its, cuts=s.cuts, dt=s.dt_used,
                            res=s.res_final) for s in steps], hist


class CPR:
    """The oracle's CPR preconditioner of one decoupled matrix."""

    def __init__(self, model: Model, Jdec, p_iters=CPR_P_ITERS, nu=CPR_NU, cf=CPR_CF):
        self.model = model
        self._J = np.ascontiguousarray(Jdec, np.float64)
        self.h = lib().orc_cpr_create(model.h, _p(self._J), p_iters, nu, cf)
        if not self.h:
            raise RuntimeError("oracle CPR: singular factor")
        self.nlevels = lib().orc_cpr_nlevels(self.h)

    def __del__(self):
        if getattr(self, "h", None) and _LIB is not None and callable(lib):
            _LIB.orc_cpr_destroy(self.h)
            self.h = None

    def level_dims(self, l):
        d = np.zeros(3, np.int32)
        n = lib().orc_cpr_level_dims(self.h, l, _ip_(d))
        return tuple(int(v) for v in d), n

    def level_dense(self, l):
        _, n = self.level_dims(l)
        out = np.zeros((n, n))
        lib().orc_cpr_level_dense(self.h, l, _p(out))
        return out

    def smooth(self, l, b, x, first):
        x = np.array(x, dtype=np.float64, order="C")
        lib().orc_cpr_smooth(self.h, l, _p(np.ascontiguousarray(b, np.float64)), _p(x), first)
        return x

    def vcycle(self, b):
        x = np.zeros(self.model.n)
        lib().orc_cpr_vcycle(self.h, _p(np.ascontiguousarray(b, np.float64)), _p(x))
        return x

    def pressure(self, rp):
        e = np.zeros(self.model.n)
        lib().orc_cpr_pressure(self.h, _p(np.ascontiguousarray(rp, np.float64)), _p(e))
        return e

    def apply(self, r):
        z = np.zeros((self.model.n, 8))
        lib().orc_cpr_apply(self.h, _p(np.ascontiguousarray(r, np.float64)), _p(z))
        return z


def zfactor(fluid, p, T, y):
    y = np.ascontiguousarray(y, np.float64)
    tcm = ctypes.c_double()
    pcm = ctypes.c_double()
    z = lib().orc_zfactor(ctypes.byref(fluid), p, T, _p(y), ctypes.byref(tcm), ctypes.byref(pcm))
    return z, tcm.value, pcm.value


def gas_viscosity(fluid, T, y):
    """Gas-phase viscosity (Pa s) of composition y[6] at T (K)."""
    y = np.ascontiguousarray(y, np.float64)
    return lib().orc_gas_viscosity(ctypes.byref(fluid), T, _p(y))
