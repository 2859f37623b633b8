"""Python binding of libisc (the C-ABI in include/isc.h).

Argument marshalling only: every step of the Newton hot path runs in the HIP
kernels of ``libisc.so``.  PyTorch supplies device memory and the stream.
The library is loaded from this package directory; if it is missing the
binding raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

from . import inputs as I

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libisc.so")
_LIB = None

ISC_OK, ISC_ERR_ARG, ISC_ERR_HIP, ISC_ERR_OOM = 0, -1, -2, -3
ISC_ERR_SINGULAR, ISC_ERR_NONFINITE, ISC_ERR_LINEAR_NOCONV, ISC_ERR_NEWTON_NOCONV = -4, -5, -6, -7
ISC_FP64, ISC_MIXED = 0, 1
ISC_PC_BILU0, ISC_PC_CPR = 0, 1
ISC_KRYLOV_GMRES, ISC_KRYLOV_BICGSTAB = 0, 1
CPR_P_ITERS = 12    # default GMRES steps of the CPR pressure solve

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_f64 = ctypes.c_double


class SolveOpts(ctypes.Structure):
    _fields_ = [("restart", _i32), ("max_restarts", _i32), ("precision", _i32), ("inner_iters", _i32),
                ("precond", _i32), ("p_iters", _i32), ("rtol", _f64), ("krylov", _i32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", _i32), ("inner_iters_total", _i32), ("restarts", _i32), ("reserved", _i32),
                ("relres_est", _f64), ("relres_true", _f64)]


class NewtonOpts(ctypes.Structure):
    _fields_ = [("lin", SolveOpts), ("tol", _f64)]


class NewtonInfo(ctypes.Structure):
    _fields_ = [("converged", _i32), ("bad_cell", _i32), ("res_scaled", _f64), ("lin", SolveInfo),
                ("ms_assemble", ctypes.c_float), ("ms_decouple", ctypes.c_float),
                ("ms_precond", ctypes.c_float), ("ms_krylov", ctypes.c_float), ("ms_update", ctypes.c_float)]


class IscError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libisc status {status}: {msg}")
        self.status = status


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1811_11992_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.isc_create.argtypes = [_vp, _vp, _vp, _f64, _vp, _vp, _i32, _vp, _vp, ctypes.POINTER(_vp)]
        L.isc_destroy.argtypes = [_vp]
        L.isc_set_params.argtypes = [_vp, _vp, _vp]
        L.isc_set_heater.argtypes = [_vp, _i32, _f64]
        L.isc_bcsr_pattern.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_i32)]
        L.isc_assemble.argtypes = [_vp, _vp, _vp, _f64, _vp, _vp]
        L.isc_decouple.argtypes = [_vp, _vp, _vp, ctypes.POINTER(_i32)]
        L.isc_solve.argtypes = [_vp, _vp, _vp, _vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo)]
        L.isc_solve_bicgstab.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_double,
                                         ctypes.POINTER(SolveInfo)]
        L.isc_newton_step.argtypes = [_vp, _vp, _vp, _f64, ctypes.POINTER(NewtonOpts), ctypes.POINTER(NewtonInfo)]
        L.isc_spmv.argtypes = [_vp, _vp, _vp, _vp]
        L.isc_bilu0.argtypes = [_vp, _vp, _vp]
        L.isc_bilu0_apply.argtypes = [_vp, _vp, _vp, _vp, _vp]
        L.isc_bilu0_apply_spmv.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
        L.isc_update.argtypes = [_vp, _vp, _vp]
        L.isc_bilu0_apply_spmv32.argtypes = [_vp, _vp, _vp, _vp, _vp]
        L.isc_cpr_pressure_solve.argtypes = [_vp, _vp, _i32, _vp, _vp]
        L.isc_cpr_apply.argtypes = [_vp, _vp, _i32, _vp, _vp, _vp]
        L.isc_scaled_norm.argtypes = [_vp, _vp, _f64, ctypes.POINTER(_f64)]
        L.isc_scaled_norm_noalloc.argtypes = [_vp, _vp, _vp, _vp, _f64, _vp, _vp]
        L.isc_adjoint.argtypes = [_vp, _vp, _vp, _f64, _vp, _f64, _vp, _vp, _vp, ctypes.POINTER(SolveOpts),
                                  ctypes.POINTER(SolveInfo)]
        L.isc_oil_rate.argtypes = [_vp, _vp, ctypes.POINTER(_f64)]
        L.isc_well_count.argtypes = [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]
        L.isc_well_state.argtypes = [_vp, _vp, _vp]
        L.isc_set_well_state.argtypes = [_vp, _vp, _vp]
        L.isc_well_controls.argtypes = [_vp, _vp, ctypes.POINTER(_i32)]
        L.isc_well_solve.argtypes = [_vp, _vp, ctypes.POINTER(_i32)]
        L.isc_well_border.argtypes = [_vp, _vp, _vp, _f64, _vp, _vp, _vp, _vp]
        L.isc_profile.argtypes = [_vp, _i32, _vp, _vp]
        L.isc_profile_vectors.argtypes = [_vp, _vp]
        L.isc_last_error.argtypes = [_vp]
        L.isc_last_error.restype = ctypes.c_char_p
        for name in ("isc_create", "isc_destroy", "isc_set_params", "isc_bcsr_pattern", "isc_assemble",
                     "isc_decouple", "isc_solve", "isc_solve_bicgstab", "isc_newton_step", "isc_spmv", "isc_bilu0",
                     "isc_bilu0_apply", "isc_bilu0_apply_spmv", "isc_update", "isc_scaled_norm", "isc_adjoint",
                     "isc_profile", "isc_profile_vectors", "isc_oil_rate", "isc_scaled_norm_noalloc",
                     "isc_cpr_pressure_solve", "isc_cpr_apply", "isc_bilu0_apply_spmv32", "isc_set_heater"):
            getattr(L, name).restype = _i32
        _LIB = L
    return _LIB


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous() and t.dtype == torch.float64, (t.device, t.dtype)
    return ctypes.c_void_p(t.data_ptr())


def solve_opts(restart=30, max_restarts=20, precision=ISC_FP64, inner_iters=0, rtol=1e-8, precond=ISC_PC_BILU0,
               p_iters=0, krylov=None) -> SolveOpts:
    return SolveOpts(restart, max_restarts, precision, inner_iters, precond, p_iters, rtol,
                     ISC_KRYLOV_GMRES if krylov is None else krylov)


def bicgstab_opts(max_iters=600, rtol=1e-8) -> SolveOpts:
    """BiCGSTAB with BILU(0) in FP64 (at most max_iters iterations, a
    multiple of 30)."""
    return solve_opts(restart=30, max_restarts=max(1, max_iters // 30), rtol=rtol, krylov=ISC_KRYLOV_BICGSTAB)


def cpr_opts(p_iters=CPR_P_ITERS, restart=30, max_restarts=20, rtol=1e-8) -> SolveOpts:
    """FP64 flexible GMRES with the CPR preconditioner."""
    return solve_opts(restart=restart, max_restarts=max_restarts, rtol=rtol, precond=ISC_PC_CPR, p_iters=p_iters)


class Context:
    """One ``isc_ctx``: a grid, its physics card, rock, wells and workspace."""

    def __init__(self, wl: I.Workload, fluid: I.Fluid | None = None, restart: int = 30,
                 inner_iters: int = 0, device: str = "cuda", cpr_p_iters: int | None = None):
        L = lib()
        self.wl = wl
        self.n = wl.ncell
        self.device = torch.device(device)
        self.fluid = fluid if fluid is not None else I.physics_card()
        self._grid = wl.grid()
        self._wells, self._keep = wl.well_structs()
        self.logk = torch.tensor(wl.logk, dtype=torch.float64, device=self.device)
        self.poro = torch.tensor(wl.poro, dtype=torch.float64, device=self.device)
        self.max_opts = solve_opts(restart=restart, inner_iters=inner_iters)
        if cpr_p_iters is not None:   # also allocate the CPR preconditioner
            self.max_opts.precond = ISC_PC_CPR
            self.max_opts.p_iters = cpr_p_iters
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = L.isc_create(ctypes.byref(self._grid), ctypes.byref(self.fluid), _ptr(self.logk), wl.kv_over_kh,
                          _ptr(self.poro), ctypes.cast(self._wells, _vp), len(wl.wells),
                          ctypes.byref(self.max_opts), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != ISC_OK:
            raise IscError(st, "isc_create failed (see stderr)")
        self.h = h
        rp, ci, nn = _vp(), _vp(), _i32()
        self._check(L.isc_bcsr_pattern(self.h, ctypes.byref(rp), ctypes.byref(ci), ctypes.byref(nn)))
        self.nnzb = nn.value
        ncw, ncp = _i32(), _i32()
        self._check(L.isc_well_count(self.h, ctypes.byref(ncw), ctypes.byref(ncp)))
        self.ncw, self.ncp = ncw.value, ncp.value

    def close(self):
        """Destroy the context now (waits for its stream, frees its workspace).
        Programs that end soon after should call it rather than leave the
        destruction to interpreter shutdown, when the HIP runtime may already
        be going away."""
        if getattr(self, "h", None) is not None and _LIB is not None:
            _LIB.isc_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _check(self, st):
        if st != ISC_OK:
            raise IscError(st, lib().isc_last_error(self.h).decode())
        return st

    def empty_F(self):
        return torch.empty((self.n, 8), dtype=torch.float64, device=self.device)

    def empty_J(self):
        return torch.empty((self.nnzb, 8, 8), dtype=torch.float64, device=self.device)

    # ---- C-ABI calls (same names as include/isc.h)
    def isc_set_params(self, logk: torch.Tensor | None = None, A=None):
        a = None if A is None else (ctypes.c_double * 4)(*[float(x) for x in A])
        if logk is not None:
            self.logk = logk.to(self.device, torch.float64).contiguous()
        self._check(lib().isc_set_params(self.h, _ptr(logk if logk is None else self.logk), a))

    def isc_set_heater(self, cell: int, rate_W: float):
        self._check(lib().isc_set_heater(self.h, int(cell), float(rate_W)))

    # ---- controlled wells (kinds 3, 4)
    def isc_well_state(self):
        """(bhp [ncw], on_limit [ncw]) as numpy arrays."""
        bhp = (ctypes.c_double * max(1, self.ncw))()
        on = (ctypes.c_int32 * max(1, self.ncw))()
        self._check(lib().isc_well_state(self.h, bhp, on))
        return np.array(bhp[:self.ncw]), np.array(on[:self.ncw], dtype=np.int32)

    def isc_set_well_state(self, bhp, on_limit):
        b = (ctypes.c_double * max(1, self.ncw))(*[float(x) for x in bhp])
        o = (ctypes.c_int32 * max(1, self.ncw))(*[int(x) for x in on_limit])
        self._check(lib().isc_set_well_state(self.h, b, o))

    def isc_well_controls(self, u):
        nsw = _i32()
        self._check(lib().isc_well_controls(self.h, _ptr(u), ctypes.byref(nsw)))
        return nsw.value

    def isc_well_solve(self, u):
        nsw = _i32()
        self._check(lib().isc_well_solve(self.h, _ptr(u), ctypes.byref(nsw)))
        return nsw.value

    def isc_well_border(self, u, u_old, dt):
        """(R [ncw], D [ncw]) numpy and (B [ncp][8], C [ncp][8]) device tensors."""
        R = (ctypes.c_double * max(1, self.ncw))()
        D = (ctypes.c_double * max(1, self.ncw))()
        B = torch.zeros((max(1, self.ncp), 8), dtype=torch.float64, device=self.device)
        C = torch.zeros((max(1, self.ncp), 8), dtype=torch.float64, device=self.device)
        self._check(lib().isc_well_border(self.h, _ptr(u), _ptr(u_old), float(dt), R, D, _ptr(B), _ptr(C)))
        return np.array(R[:self.ncw]), np.array(D[:self.ncw]), B[:self.ncp], C[:self.ncp]

    def isc_assemble(self, u, u_old, dt, F=None, J=None):
        F = self.empty_F() if F is None else F
        J = self.empty_J() if J is None else J
        self._check(lib().isc_assemble(self.h, _ptr(u), _ptr(u_old), dt, _ptr(F), _ptr(J)))
        return F, J

    def isc_decouple(self, J, F):
        bad = _i32(-1)
        st = lib().isc_decouple(self.h, _ptr(J), _ptr(F), ctypes.byref(bad))
        if st == ISC_ERR_SINGULAR:
            return st, bad.value
        self._check(st)
        return st, bad.value

    def isc_solve(self, Jdec, b, opts: SolveOpts | None = None, x=None, check=True):
        x = torch.empty_like(b) if x is None else x
        info = SolveInfo()
        st = lib().isc_solve(self.h, _ptr(Jdec), _ptr(b), _ptr(x), ctypes.byref(opts or solve_opts()),
                             ctypes.byref(info))
        if check:
            self._check(st)
        return x, info, st

    def isc_solve_bicgstab(self, Jdec, b, max_iters=1000, rtol=1e-8, x=None, check=True):
        x = torch.empty_like(b) if x is None else x
        info = SolveInfo()
        st = lib().isc_solve_bicgstab(self.h, _ptr(Jdec), _ptr(b), _ptr(x), max_iters, rtol, ctypes.byref(info))
        if check:
            self._check(st)
        return x, info, st

    def isc_newton_step(self, u, u_old, dt, tol=1e-10, lin: SolveOpts | None = None):
        o = NewtonOpts(lin or solve_opts(), tol)
        info = NewtonInfo()
        st = lib().isc_newton_step(self.h, _ptr(u), _ptr(u_old), dt, ctypes.byref(o), ctypes.byref(info))
        return st, info

    def isc_spmv(self, Jdec, x, y=None):
        y = torch.empty_like(x) if y is None else y
        self._check(lib().isc_spmv(self.h, _ptr(Jdec), _ptr(x), _ptr(y)))
        return y

    def isc_bilu0(self, Jdec, Dinv=None):
        Dinv = torch.empty((self.n, 8, 8), dtype=torch.float64, device=self.device) if Dinv is None else Dinv
        self._check(lib().isc_bilu0(self.h, _ptr(Jdec), _ptr(Dinv)))
        return Dinv

    def isc_bilu0_apply(self, Jdec, Dinv, r, z=None):
        z = torch.empty_like(r) if z is None else z
        self._check(lib().isc_bilu0_apply(self.h, _ptr(Jdec), _ptr(Dinv), _ptr(r), _ptr(z)))
        return z

    def isc_bilu0_apply_spmv(self, Jdec, Dinv, r, z=None, w=None):
        z = torch.empty_like(r) if z is None else z
        w = torch.empty_like(r) if w is None else w
        self._check(lib().isc_bilu0_apply_spmv(self.h, _ptr(Jdec), _ptr(Dinv), _ptr(r), _ptr(z), _ptr(w)))
        return z, w

    def isc_bilu0_apply_spmv32(self, Jdec, r, z=None, w=None):
        z = torch.empty_like(r) if z is None else z
        w = torch.empty_like(r) if w is None else w
        self._check(lib().isc_bilu0_apply_spmv32(self.h, _ptr(Jdec), _ptr(r), _ptr(z), _ptr(w)))
        return z, w

    def isc_cpr_pressure_solve(self, Jdec, rp, p_iters=CPR_P_ITERS, e=None):
        e = torch.empty_like(rp) if e is None else e
        self._check(lib().isc_cpr_pressure_solve(self.h, _ptr(Jdec), p_iters, _ptr(rp), _ptr(e)))
        return e

    def isc_cpr_apply(self, Jdec, r, p_iters=CPR_P_ITERS, z=None, w=None):
        z = torch.empty_like(r) if z is None else z
        w = torch.empty_like(r) if w is None else w
        self._check(lib().isc_cpr_apply(self.h, _ptr(Jdec), p_iters, _ptr(r), _ptr(z), _ptr(w)))
        return z, w

    def isc_update(self, u, du):
        return lib().isc_update(self.h, _ptr(u), _ptr(du))

    def isc_scaled_norm(self, F, dt):
        r = _f64()
        self._check(lib().isc_scaled_norm(self.h, _ptr(F), dt, ctypes.byref(r)))
        return r.value

    def isc_adjoint(self, u_n, u_nm1, dt_n, lam_np1, dt_np1, lam_n, g_logk, g_A, opts: SolveOpts | None = None):
        """One backward step; g_logk (device) and the returned g_A are accumulated."""
        info = SolveInfo()
        a = (ctypes.c_double * 4)(*[float(x) for x in g_A])
        o = opts or solve_opts(restart=30, max_restarts=200, rtol=1e-12)
        st = lib().isc_adjoint(self.h, _ptr(u_n), _ptr(u_nm1), dt_n, _ptr(lam_np1), dt_np1, _ptr(lam_n),
                               _ptr(g_logk), a, ctypes.byref(o), ctypes.byref(info))
        self._check(st)
        return [a[k] for k in range(4)], info

    def isc_oil_rate(self, u):
        q = _f64()
        self._check(lib().isc_oil_rate(self.h, _ptr(u), ctypes.byref(q)))
        return q.value


NOALLOC_MAX_CELLS = 16777216   # ISC_NOALLOC_MAX_CELLS


def isc_scaled_norm_noalloc(grid: I.Grid, fluid: I.Fluid, poro: torch.Tensor, F: torch.Tensor, dt: float,
                            res: torch.Tensor, stream: "torch.cuda.Stream | None" = None) -> int:
    """Context-free, allocation-free scaled max-norm of F into res[0] (device),
    enqueued on `stream` (default: the current stream).  Returns the status;
    on error lib().isc_last_error(None) holds the message."""
    s = stream if stream is not None else torch.cuda.current_stream(res.device)
    return lib().isc_scaled_norm_noalloc(ctypes.byref(grid), ctypes.byref(fluid), _ptr(poro), _ptr(F), dt,
                                         _ptr(res), ctypes.c_void_p(s.cuda_stream))


PROF_CLASSES = ("spmv", "ilu_apply", "assemble", "decouple", "ilu_factor", "krylov", "cpr_pressure", "cpr_setup",
                "ilu_spmv", "ilu_spmv32")


def _profile_call(ctx, enable):
    ms = (ctypes.c_double * len(PROF_CLASSES))()      # ISC_PROF_NCLASS entries
    cnt = (ctypes.c_int32 * len(PROF_CLASSES))()
    ctx._check(lib().isc_profile(ctx.h, enable, ms, cnt))
    return {name: (ms[k], cnt[k]) for k, name in enumerate(PROF_CLASSES)}


def isc_profile(ctx: "Context", enable: int):
    """Start (1), stop (0) or read (-1) the library's kernel-class timers;
    returns {class: (milliseconds, launches)}."""
    return _profile_call(ctx, enable)


def isc_profile_vectors(ctx: "Context"):
    """{class: full-length vectors streamed beyond the class's fixed access
    pattern} over the current profiling window (the Gram-Schmidt update
    folded into the FP64 GMRES iteration's forward sweep)."""
    vec = (ctypes.c_double * len(PROF_CLASSES))()
    ctx._check(lib().isc_profile_vectors(ctx.h, vec))
    return {name: vec[k] for k, name in enumerate(PROF_CLASSES)}


class Simulator:
    """Implicit-Euler time loop driving ``isc_newton_step``; on a failed step
    the step size is halved and the step retried (at most four times)."""

    def __init__(self, ctx: Context, tol=1e-10, max_newton=12, lin: SolveOpts | None = None):
        self.ctx, self.tol, self.max_newton = ctx, tol, max_newton
        self.lin = lin or solve_opts()

    def step(self, u, dt):
        """Advance u (in place) by one step of at most dt; returns a record.
        Each attempt starts with the controlled wells' step-start control
        check; a failed attempt restores u and the well state."""
        u_old = u.clone()
        dts, cuts = dt, 0
        rec = dict(newton=0, lin=0, inner=0, cuts=0)
        wells0 = self.ctx.isc_well_state() if self.ctx.ncw else None
        while True:
            ok = False
            nit = 0
            if wells0 is not None:
                self.ctx.isc_well_controls(u)
            for nit in range(self.max_newton + 1):
                st, info = self.ctx.isc_newton_step(u, u_old, dts, self.tol, self.lin)
                rec["lin"] += info.lin.iters
                rec["inner"] += info.lin.inner_iters_total
                if st != ISC_OK:
                    break
                if info.converged:
                    ok = True
                    break
            else:
                nit += 1   # every call updated u: max_newton + 1 iterations, none converged
            rec["newton"] += nit
            rec["res"] = info.res_scaled
            if ok:
                rec.update(cuts=cuts, dt=dts)
                return rec
            u.copy_(u_old)
            if wells0 is not None:
                self.ctx.isc_set_well_state(*wells0)
            cuts += 1
            dts *= 0.5
            if cuts > 4:
                raise IscError(ISC_ERR_NEWTON_NOCONV, f"Newton failed after {cuts - 1} step cuts")

    def run(self, u0, dt, nsteps, history=False):
        u = u0.clone()
        recs, hist = [], [u.clone()] if history else None
        for _ in range(nsteps):
            recs.append(self.step(u, dt))
            if history:
                hist.append(u.clone())
        return u, recs, hist


def __getattr__(name):
    """isc.OilProduction: the differentiation form (adjoint.py), imported on
    first use."""
    if name == "OilProduction":
        from .adjoint import OilProduction
        return OilProduction
    raise AttributeError(f"module {__name__!r} has no attribute {name!r}")
