"""Benchmark: cells x Newton-iterations per second of the whole hot path
(assemble -> convergence check -> Gauss-Jordan decoupling -> BILU(0) ->
GMRES(30) to 1e-8 -> safeguarded update) on one MI355X.

A step is one Newton iteration that solves; when Newton has converged the
next timestep starts (the converged-check assembly is inside the timed
region, counted as no step).  Inputs are resident in HBM before timing.
The JSON line's value is the chosen precision on the chosen workload;
unless --no-forms, it also carries the other precision on the same workload
(precision form: FP32 BILU(0) and inner SpMV inside FP64 FGMRES) and the
cost of the differentiation form (forward and backward ms per step of the
adjoint of cumulative oil production on the 60x60x10 grid).

    python bench.py [--steps K] [--warmup W] [--workload C3] [--precision fp64|mixed]
                    [--precond bilu0|cpr] [--p-iters 8]

Unless --no-forms, a third leg runs the FP64 solve with the CPR two-stage
preconditioner (pressure multigrid + BILU(0), in FP64 flexible GMRES) on the
same workload and window.  The default window (5 warm-up, 20 timed Newton
iterations) is the one the benchmark is quoted on.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
METRIC = "cells·Newton-its/s (assemble+decouple+solve), FP64 vs mixed at 1e-8 rel"
UNIT = "cells·Newton-its/s"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--precision", default="fp64", choices=("fp64", "mixed"))
    ap.add_argument("--precond", default="bilu0", choices=("bilu0", "cpr"))
    ap.add_argument("--krylov", default="gmres", choices=("gmres", "bicgstab"),
                    help="Krylov method (bicgstab: FP64 with BILU(0))")
    ap.add_argument("--inner", type=int, default=12, help="FP32 inner iterations (mixed)")
    ap.add_argument("--p-iters", type=int, default=12, help="pressure GMRES steps per CPR application")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the other precision and the adjoint-cost legs")
    ap.add_argument("--cpu-layers", type=int, default=4, help="layers of the workload in the oracle sample")
    ap.add_argument("--cpu-workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="concurrent oracle processes of the all-core CPU figure (0 or 1: none)")
    ap.add_argument("--cpu-worker", type=float, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--reference-copy", type=int, default=0, metavar="MB",
                    help="first copy MB megabytes device to device ten times: the kernel of known bytes that "
                         "scales the HBM counters of a profiled run")
    return ap.parse_args()


def algorithmic_bytes(n, nnzb):
    """Bytes each kernel class must move per launch (every matrix block and
    vector element once; a neighbour's vector block re-read by another row is
    counted as a cache hit)."""
    off64 = (nnzb - n) * 64 * 8             # off-diagonal blocks of the decoupled matrix, FP64
    vec64 = n * 8 * 8                       # one FP64 block vector
    return {
        # y = A x: off-diagonal blocks + x + y
        "spmv": off64 + 2 * vec64,
        # forward + backward sweep of M = (I + L D^-1)(D + U): every
        # off-diagonal block once (L D^-1 forward, U backward), D^-1 once,
        # r read, y write, y read, z write
        "ilu_apply": off64 + n * 64 * 8 + 4 * vec64,
        # the same in FP32 storage (precision form)
        "ilu_apply32": (off64 + n * 64 * 8 + 4 * vec64) // 2,
        "spmv32": (off64 + 2 * vec64) // 2,
        # the GMRES iteration's w = A M^-1 u: BILU(0) apply and SpMV in one
        # pass.  The backward sweep already forms U z, so it publishes
        # z + U z (write) and the SpMV adds L z: the lower blocks (half the
        # off-diagonal blocks), z read, z + U z read, w write.  The Gram-
        # Schmidt update folded into the forward sweep adds j + 2 vectors at
        # iteration j, counted per launch from the library's tally.
        "ilu_spmv": (off64 + n * 64 * 8 + 4 * vec64) + (off64 // 2 + 4 * vec64),
        # the same in FP32 storage (the precision form's inner iteration, its
        # folded Gram-Schmidt update counted like the FP64 one)
        "ilu_spmv32": ((off64 + n * 64 * 8 + 4 * vec64) + (off64 // 2 + 4 * vec64)) // 2,
        # u, u_old, porosity, 3 transmissibilities in; F and J out
        "assemble": 2 * vec64 + n * 8 * 4 + vec64 + nnzb * 64 * 8,
    }


HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_PROFILE = os.path.join(HERE, "profiles", "bilu0_sweeps_200x200x50_traffic.md")


def sweep_source_hash():
    h = hashlib.sha256()
    for f in ("precond.hip", "common.h", "krylov.hip", "api.hip"):
        with open(os.path.join(HERE, "paper_1811_11992_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed counter summary, or None when
    it covers another kernel or workload or the sweep source has changed
    since the counters were taken."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            for line in fh:
                if line.startswith("traffic_record:"):
                    rec = json.loads(line.split(":", 1)[1])
                    if (rec["kernel"] == kernel and rec["workload"] == workload
                            and rec["source_sha256"] == sweep_source_hash()):
                        return rec["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    return None


class Driver:
    """Advances the simulation one solving Newton iteration at a time."""

    def __init__(self, ctx, wl, lin, tol=1e-10, max_newton=12):
        import torch
        self.ctx, self.wl, self.lin, self.tol, self.max_newton = ctx, wl, lin, tol, max_newton
        self.u = torch.tensor(wl.u0, dtype=torch.float64, device="cuda")
        self.u_old = self.u.clone()
        self.dt = wl.dt
        self.ni_in_step = 0
        self.ni = 0
        self.lin_its = 0
        self.inner_its = 0
        self.steps_done = 0
        self.cuts = 0
        self.lin_each = []       # Krylov iterations of every solving Newton iteration

    def newton_iteration(self):
        from paper_1811_11992_amd import isc
        while True:
            st, info = self.ctx.isc_newton_step(self.u, self.u_old, self.dt, self.tol, self.lin)
            if st == isc.ISC_OK and info.converged:
                self.u_old.copy_(self.u)       # next timestep
                self.steps_done += 1
                self.ni_in_step = 0
                self.dt = self.wl.dt
                continue
            if st == isc.ISC_OK and self.ni_in_step < self.max_newton:
                self.ni += 1
                self.ni_in_step += 1
                self.lin_its += info.lin.iters
                self.inner_its += info.lin.inner_iters_total
                self.lin_each.append(info.lin.iters)
                return info
            # failed step: restore and halve the step
            self.u.copy_(self.u_old)
            self.dt *= 0.5
            self.cuts += 1
            self.ni_in_step = 0
            if self.cuts > 40:
                raise RuntimeError(f"too many step cuts (status {st})")


def host_cpu():
    """The host's CPU model and logical core count (the oracle uses one)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "host_logical_cpus": os.cpu_count()}


def cpu_sample(wl, layers, start_at=None):
    """One Newton iteration of the oracle, as it stands, on the top `layers`
    layers of the workload: (cells, seconds, GMRES iterations, status, start
    and end wall-clock times).  With start_at, the iteration starts at that
    wall-clock time (so that concurrent samples overlap)."""
    import oracle as O
    from paper_1811_11992_amd import inputs as I
    nxy = wl.nx * wl.ny
    n = nxy * layers
    sub = I.Workload(name=wl.name + f"-top{layers}", nx=wl.nx, ny=wl.ny, nz=layers, dx=wl.dx, dy=wl.dy, dz=wl.dz,
                     logk=wl.logk[:n].copy(), kv_over_kh=wl.kv_over_kh, poro=wl.poro[:n].copy(),
                     wells=[dict(w, cells=[c for c in w["cells"] if c < n]) for w in wl.wells],
                     u0=wl.u0[:, :n].copy(), dt=wl.dt, nsteps=1, seed=wl.seed)
    sub.wells = [w for w in sub.wells if w["cells"]]
    m = O.Model(sub)
    if start_at is not None:
        time.sleep(max(0.0, start_at - time.time()))
    w0 = time.time()
    t0 = time.perf_counter()
    st, u, info = m.newton_step(sub.u0, sub.u0, sub.dt)
    el = time.perf_counter() - t0
    return n, el, int(info.iters_lin), int(st), w0, time.time()


def cpu_baseline(wl, layers, workers=0):
    """The oracle, as it stands, on a bounded sample of the workload (one
    Newton iteration on its top `layers` layers), in this process (one core);
    with workers > 1 also the same sample in that many concurrent
    single-threaded processes, for the throughput of all the host's cores."""
    n, el, its, st, _, _ = cpu_sample(wl, layers)
    out = {"value": n / el, "unit": UNIT, "cores": 1, "kind": "oracle", **host_cpu(),
           "sample": f"one Newton iteration (assemble, decouple, BILU(0)-GMRES(30) to 1e-8, update) of the "
                     f"serial FP64 oracle on the top {layers} layers of {wl.name} ({n} cells), first step "
                     f"from the initial state; {its} GMRES iterations, {el:.1f} s",
           "status": st}
    if workers > 1:
        import subprocess
        start_at = time.time() + 20.0
        cmd = [sys.executable, os.path.abspath(__file__), "--cpu-worker", str(start_at), "--workload", wl.name,
               "--cpu-layers", str(layers)]
        procs = [subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True)
                 for _ in range(workers)]
        recs = []
        for p in procs:
            o, _ = p.communicate(timeout=600)
            line = [x for x in o.splitlines() if x.startswith("{")]
            if p.returncode == 0 and line:
                recs.append(json.loads(line[-1]))
        if len(recs) == workers:
            span = max(r["end"] for r in recs) - min(r["start"] for r in recs)
            out["all_cores"] = {"value": sum(r["cells"] for r in recs) / span, "unit": UNIT, "cores": workers,
                                "wall_s": round(span, 2),
                                "sample": f"the same sample in {workers} concurrent single-threaded processes, "
                                          f"started together; cells of all of them over the span from the first "
                                          f"start to the last end"}
    return out


def run_newton(wl, precision, inner, warmup, steps, precond="bilu0", p_iters=8, krylov="gmres"):
    """Times `steps` solving Newton iterations; returns (rate, seconds,
    statistics, class profile, extra-vector tally)."""
    import torch
    from paper_1811_11992_amd import isc
    mixed = precision == "mixed"
    cpr = precond == "cpr"
    ctx = isc.Context(wl, restart=30, inner_iters=inner if mixed else 0, cpr_p_iters=p_iters if cpr else None)
    if krylov == "bicgstab":
        lin = isc.bicgstab_opts(max_iters=600, rtol=1e-8)
    elif cpr:
        lin = isc.cpr_opts(p_iters=p_iters, restart=30, max_restarts=20, rtol=1e-8)
    else:
        lin = isc.solve_opts(restart=30, max_restarts=20, rtol=1e-8,
                             precision=isc.ISC_MIXED if mixed else isc.ISC_FP64, inner_iters=inner if mixed else 0)
    drv = Driver(ctx, wl, lin)
    for _ in range(warmup):
        drv.newton_iteration()
    torch.cuda.synchronize()
    ni0, lin0, inner0 = drv.ni, drv.lin_its, drv.inner_its
    steps0 = drv.steps_done
    isc.isc_profile(ctx, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        drv.newton_iteration()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = isc.isc_profile(ctx, 0)
    vec = isc.isc_profile_vectors(ctx)
    stats = {"gmres_its_per_newton": round((drv.lin_its - lin0) / max(1, drv.ni - ni0), 2),
             "inner_its_per_newton": round((drv.inner_its - inner0) / max(1, drv.ni - ni0), 2),
             "gmres_its_each": drv.lin_each[ni0:],
             "timesteps_completed": drv.steps_done, "timesteps_completed_in_window": drv.steps_done - steps0,
             "step_cuts": drv.cuts, "nnzb": ctx.nnzb}
    ctx.close()
    del drv, ctx
    gc.collect()
    torch.cuda.synchronize()
    return wl.ncell * steps / el, el, stats, prof, vec


def adjoint_cost(name="C4", nsteps=20, every=5):
    """Differentiation form: one forward run (checkpoints every `every` steps)
    and its backward pass (segment recomputation + one adjoint solve per
    step) of cumulative oil production on `name`; times per step."""
    import torch
    from paper_1811_11992_amd import inputs as I
    from paper_1811_11992_amd import isc
    from paper_1811_11992_amd.adjoint import OilProduction, log_frequency_factors
    wl = I.make_workload(name)
    fl = I.physics_card()
    ctx = isc.Context(wl, fluid=fl)
    u0 = torch.tensor(wl.u0, dtype=torch.float64, device="cuda")
    logk = torch.tensor(wl.logk, dtype=torch.float64, device="cuda").requires_grad_(True)
    lnA = log_frequency_factors(fl).requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = OilProduction.apply(logk, lnA, ctx, u0, wl.dt, nsteps, every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ok = bool(torch.isfinite(logk.grad).all()) and bool(torch.isfinite(lnA.grad).all())
    ctx.close()
    del ctx, J
    gc.collect()
    return {"workload": f"{name}: {wl.nx}x{wl.ny}x{wl.nz}, {nsteps} steps, checkpoints every {every}",
            "forward_ms_per_step": round((t1 - t0) / nsteps * 1e3, 2),
            "backward_ms_per_step": round((t2 - t1) / nsteps * 1e3, 2),
            "backward_over_forward": round((t2 - t1) / (t1 - t0), 3),
            "gradient_finite": ok}


def bicgstab_cost(name="C3", reps=2):
    """The paper's Krylov method beside GMRES(30) on the benchmark's first
    linear system: the decoupled system of the first Newton iteration, both
    with BILU(0) (factor included), FP64, to 1e-8.  Iterations, true relative
    residual and wall time of the last of `reps` solves of each.  Not part of
    the default run; call it as bench.bicgstab_cost()."""
    import torch
    from paper_1811_11992_amd import inputs as I
    from paper_1811_11992_amd import isc
    wl = I.make_workload(name)
    ctx = isc.Context(wl)
    u = torch.tensor(wl.u0, dtype=torch.float64, device="cuda")
    F, J = ctx.isc_assemble(u, u, wl.dt)
    ctx.isc_decouple(J, F)
    b = -F
    out = {"workload": f"{name}: {wl.nx}x{wl.ny}x{wl.nz}, first Newton iteration's decoupled system",
           "cells": wl.ncell}
    for label in ("gmres30", "bicgstab"):
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if label == "gmres30":
                x, info, st = ctx.isc_solve(J, b, isc.solve_opts(rtol=1e-8))
            else:
                x, info, st = ctx.isc_solve_bicgstab(J, b, rtol=1e-8)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
        out[label] = {"iters": info.iters, "relres_true": info.relres_true, "ms": round((t1 - t0) * 1e3, 2)}
    ctx.close()
    del ctx
    gc.collect()
    return out


def wells_cost(name="C3", nsteps=1, cpr=False, p_iters=12):
    """The workload with its wells as controlled wells (bhp unknowns): the
    injector column holding its air rate up to P0 + 5 MPa, the producer column
    holding a total molar rate of half of it down to 0.8 P0; `nsteps` implicit
    steps of FP64 BILU(0)-GMRES(30) (with cpr: FP64 flexible GMRES(30) with
    CPR, p_iters pressure GMRES steps) with the time loop; ms and Krylov
    iterations per Newton iteration and the final well state.  Not part of
    the default run; call it as bench.wells_cost() (under a kernel trace for
    the well kernels' share)."""
    import torch
    from paper_1811_11992_amd import inputs as I
    from paper_1811_11992_amd import isc
    wl = I.make_workload(name)
    inj, prod = wl.wells[0], wl.wells[1]
    wl.wells = [dict(inj, kind=I.WELL_INJECTOR, control=I.CTRL_RATE, limit=I.P0 + 5.0e6),
                dict(kind=I.WELL_PRODUCER, cells=prod["cells"], target=0.5 * inj["target"],
                     control=I.CTRL_TOTAL, limit=0.8 * I.P0)]
    if cpr:
        ctx = isc.Context(wl, cpr_p_iters=p_iters)
        lin = isc.cpr_opts(p_iters=p_iters, rtol=1e-8)
    else:
        ctx = isc.Context(wl)
        lin = isc.solve_opts(rtol=1e-8)
    sim = isc.Simulator(ctx, tol=1e-10, lin=lin)
    u = torch.tensor(wl.u0, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [sim.step(u, wl.dt) for _ in range(nsteps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    nit = sum(r["newton"] for r in recs)
    bhp, on = ctx.isc_well_state()
    out = {"workload": f"{name} with controlled wells, {nsteps} step(s)", "solver": "cpr" if cpr else "bilu0",
           "newton": nit,
           "ms_per_newton": round(el / max(1, nit) * 1e3, 1),
           "krylov_per_newton": round(sum(r["lin"] for r in recs) / max(1, nit), 1),
           "cuts": sum(r["cuts"] for r in recs), "bhp": bhp.tolist(), "on_limit": on.tolist()}
    ctx.close()
    del ctx
    gc.collect()
    return out


def precision_steps(name="C3", nsteps=10, inner=12):
    """The precision form against FP64, step by step: `nsteps` implicit steps
    of the workload run twice from the same initial state, by FP64
    BILU(0)-GMRES(30) and by the precision form (FP32 inner GMRES, m_in =
    inner), each with the time loop's step cuts; per step the largest
    relative state difference (per unknown, scaled by max(|u|, floor)), both
    runs' Newton iterations and step sizes.  Not part of the default run; call
    it as bench.precision_steps()."""
    import torch
    from paper_1811_11992_amd import inputs as I
    from paper_1811_11992_amd import isc
    wl = I.make_workload(name)
    ctx = isc.Context(wl, restart=30, inner_iters=inner)
    lins = {"fp64": isc.solve_opts(rtol=1e-8),
            "mixed": isc.solve_opts(rtol=1e-8, precision=isc.ISC_MIXED, inner_iters=inner)}
    sims = {k: isc.Simulator(ctx, tol=1e-10, lin=v) for k, v in lins.items()}
    states = {k: torch.tensor(wl.u0, dtype=torch.float64, device="cuda") for k in lins}
    floor = torch.tensor([1.0, 1, 1, 1, 1, 1, 1, 5000.0], dtype=torch.float64, device="cuda")
    steps = []
    for s in range(nsteps):
        rec = {}
        for k in lins:
            r = sims[k].step(states[k], wl.dt)
            rec[k] = {"newton": r["newton"], "dt": r["dt"], "cuts": r["cuts"]}
        d = (states["mixed"] - states["fp64"]).abs().amax(dim=1)
        scale = torch.maximum(states["fp64"].abs().amax(dim=1), floor)
        rec["state_rel_diff"] = float((d / scale).max())
        steps.append(rec)
        note(f"{name} step {s + 1}: {rec}")
    ctx.close()
    del ctx
    gc.collect()
    return {"workload": f"{name}: {wl.nx}x{wl.ny}x{wl.nz}, {nsteps} steps, FP64 vs precision form (m_in {inner})",
            "steps": steps, "max_state_rel_diff": max(x["state_rel_diff"] for x in steps)}


def scale_leg(name="C5", nsteps=10, every=5, inner=12, dt_days=0.0125, p_iters=12):
    """The precision and differentiation forms at the largest configured
    size: `nsteps` implicit steps of `dt_days` of the precision form (FP32
    BILU(0) and inner SpMV in FP64 FGMRES(30)), then the gradient of
    cumulative oil production over those steps (checkpoints every `every`
    steps; the forward steps and the recomputed segments solved in FP64 with
    the CPR preconditioner, one FP64 adjoint solve per step).  Reports device
    memory (the context, and the peak of the whole leg), wall time per step
    of each pass and the Newton and Krylov counts.  Not part of the default
    run; call it as bench.scale_leg()."""
    import torch
    from paper_1811_11992_amd import inputs as I
    from paper_1811_11992_amd import isc
    from paper_1811_11992_amd.adjoint import OilProduction, log_frequency_factors
    wl = I.make_workload(name)
    fl = I.physics_card()
    torch.cuda.synchronize()
    free0, total = torch.cuda.mem_get_info()
    dt = dt_days * 86400.0
    ctx = isc.Context(wl, fluid=fl, restart=30, inner_iters=inner, cpr_p_iters=p_iters)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    lin = isc.solve_opts(restart=30, max_restarts=20, rtol=1e-8, precision=isc.ISC_MIXED, inner_iters=inner)
    sim = isc.Simulator(ctx, tol=1e-10, lin=lin)
    u = torch.tensor(wl.u0, dtype=torch.float64, device="cuda")
    steps = []
    free_min = free1

    def progress(msg):
        print(f"{name}: {msg}", file=sys.stderr, flush=True)

    progress(f"context holds {(free0 - free1) / 2**30:.1f} GiB")
    for _ in range(nsteps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec = sim.step(u, dt)
        torch.cuda.synchronize()
        steps.append({"ms": round((time.perf_counter() - t0) * 1e3, 1), "newton": rec["newton"],
                      "outer": rec["lin"], "inner": rec["inner"], "cuts": rec["cuts"]})
        free_min = min(free_min, torch.cuda.mem_get_info()[0])
        progress(f"precision-form step {len(steps)}: {steps[-1]}")
    # the differentiation form over the same steps (its forward pass runs the
    # FP64 solver in parity mode, as the gradient needs)
    logk = torch.tensor(wl.logk, dtype=torch.float64, device="cuda").requires_grad_(True)
    lnA = log_frequency_factors(fl).requires_grad_(True)
    u0 = torch.tensor(wl.u0, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = OilProduction.apply(logk, lnA, ctx, u0, dt, nsteps, every, 1e-10, progress,
                            isc.cpr_opts(p_iters=p_iters))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    free_min = min(free_min, torch.cuda.mem_get_info()[0])
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    free_min = min(free_min, torch.cuda.mem_get_info()[0])
    ok = bool(torch.isfinite(logk.grad).all()) and bool(torch.isfinite(lnA.grad).all())
    out = {"workload": f"{name}: {wl.nx}x{wl.ny}x{wl.nz} ({wl.ncell} cells), {nsteps} steps of {dt_days} day",
           "device_memory_GiB": {"context": round((free0 - free1) / 2**30, 2),
                                 "peak_in_use": round((free0 - free_min) / 2**30, 2),
                                 "device_total": round(total / 2**30, 1)},
           "precision_form_steps": steps,
           "precision_form_ms_per_step": round(sum(x["ms"] for x in steps) / nsteps, 1),
           "adjoint": {"forward_ms_per_step": round((t1 - t0) / nsteps * 1e3, 1),
                       "backward_ms_per_step": round((t2 - t1) / nsteps * 1e3, 1),
                       "checkpoints_every": every, "gradient_finite": ok}}
    ctx.close()
    del ctx, J
    gc.collect()
    return out


def launch_bytes(nbytes, prof, vec, n):
    """Algorithmic bytes per launch of each class: the fixed pattern plus
    the average number of extra full-length vectors per launch that the
    library tallied (isc_profile_vectors), in the class's precision."""
    out = dict(nbytes)
    for k, v in vec.items():
        cnt = prof.get(k, (0, 0))[1]
        if k in out and cnt > 0 and v > 0:
            elem = 4 if k.endswith("32") else 8
            out[k] = out[k] + int(round(v / cnt * n * 8 * elem))
    return out


def roofline(prof, nbytes, workload):
    dom = max((k for k in nbytes if prof.get(k, (0, 0))[1] > 0), key=lambda k: prof[k][0])
    ms, cnt = prof[dom]
    achieved = nbytes[dom] / (ms / cnt * 1e-3) / 1e9
    out = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": measured_traffic(dom, workload),
           "bytes_per_launch": nbytes[dom], "avg_launch_ms": round(ms / cnt, 4)}
    # the other classes held to the 60%-of-HBM target, in the same algorithmic bytes
    others = {}
    for k in ("assemble", "spmv"):
        if k != dom and k in nbytes and prof.get(k, (0, 0))[1] > 0 and prof[k][0] > 0:
            m2, c2 = prof[k]
            others[k] = round(nbytes[k] / (m2 / c2 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    if others:
        out["frac_other_classes"] = others
        out["frac_target"] = 0.6
    return out


def classes_of(prof, nbytes):
    out = {}
    for k, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        rec = {"ms": round(ms, 3), "launches": cnt}
        if k in nbytes and ms > 0:
            rec["GB_s"] = round(nbytes[k] * cnt / (ms * 1e-3) / 1e9, 1)
        out[k] = rec
    return out


def copy_peak_gbs(nbytes=1 << 30, reps=10):
    """Achievable HBM bandwidth on this GPU: a plain device-to-device copy of
    nbytes (read + written), the best of reps, timed with events."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    del src, dst
    return 2 * nbytes / (best * 1e-3) / 1e9


def note(msg):
    """A progress line on stderr (the JSON line stays alone on stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    a = parse()
    if a.cpu_worker is not None:   # one process of the all-core CPU figure (no GPU)
        from paper_1811_11992_amd import inputs as I
        n, el, its, st, w0, w1 = cpu_sample(I.make_workload(a.workload), a.cpu_layers, a.cpu_worker)
        print(json.dumps({"cells": n, "seconds": el, "gmres": its, "status": st, "start": w0, "end": w1}),
              flush=True)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only: the hot path is built and measured on a single MI355X "
              f"(how it would shard is described in the design notes); got --gpus {a.gpus}", file=sys.stderr)
        sys.exit(2)
    from paper_1811_11992_amd import inputs as I

    if a.reference_copy > 0:
        import torch
        src = torch.ones(a.reference_copy * 1_000_000 // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    wl = I.make_workload(a.workload)
    n = wl.ncell
    if a.precond == "cpr" and a.precision != "fp64":
        print("the CPR preconditioner runs in FP64 only", file=sys.stderr)
        sys.exit(2)
    if a.krylov == "bicgstab" and (a.precision != "fp64" or a.precond != "bilu0"):
        print("BiCGSTAB runs in FP64 with BILU(0) only", file=sys.stderr)
        sys.exit(2)
    note(f"{wl.name}: {a.precision} {a.precond} {a.krylov}, {a.warmup} + {a.steps} Newton iterations")
    copy_gbs = copy_peak_gbs()
    value, el, stats, prof, vec = run_newton(wl, a.precision, a.inner, a.warmup, a.steps, a.precond, a.p_iters,
                                             a.krylov)
    base_bytes = algorithmic_bytes(n, stats["nnzb"])
    nbytes = launch_bytes(base_bytes, prof, vec, n)
    mixed = a.precision == "mixed"
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": el / a.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if not mixed else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.nx}x{wl.ny}x{wl.nz} cells, "
                               + ("FP32 BILU(0) + inner SpMV in FP64 FGMRES(30)" if mixed
                                  else f"FP64 CPR (pressure multigrid, {a.p_iters} steps) + BILU(0) in FGMRES(30)"
                                  if a.precond == "cpr" else "FP64 BILU(0)-BiCGSTAB" if a.krylov == "bicgstab"
                                  else "FP64 BILU(0)-GMRES(30)") + " to 1e-8, Newton 1e-10",
                   "cells": n, "precision": a.precision, "newton_its_timed": a.steps,
                   **{k: v for k, v in stats.items() if k != "nnzb"}},
        "roofline": roofline(prof, nbytes, wl.name),
        "kernel_classes": classes_of(prof, nbytes),
    }
    # the same achieved rate against what a plain copy reaches on this GPU
    out["roofline"]["copy_GB_s_measured"] = round(copy_gbs, 1)
    out["roofline"]["frac_of_copy"] = round(out["roofline"]["achieved"] / copy_gbs, 4)
    if not a.no_forms and a.precond == "bilu0" and a.krylov == "gmres":
        other = "fp64" if mixed else "mixed"
        note(f"{wl.name}: the {other} form")
        v2, el2, st2, prof2, vec2 = run_newton(wl, other, a.inner, a.warmup, a.steps)
        nbytes2 = launch_bytes(base_bytes, prof2, vec2, n)
        out["precision_forms"] = {
            other: {"value": v2, "ms_per_step": el2 / a.steps * 1e3,
                    **{k: v for k, v in st2.items() if k != "nnzb"},
                    "roofline": roofline(prof2, nbytes2, wl.name), "kernel_classes": classes_of(prof2, nbytes2)},
            "mixed_over_fp64": (v2 / value) if not mixed else (value / v2),
        }
        note("C4: adjoint cost")
        out["adjoint"] = adjoint_cost()
        note(f"{wl.name}: CPR")
        v3, el3, st3, prof3, vec3 = run_newton(wl, "fp64", a.inner, a.warmup, a.steps, "cpr", a.p_iters)
        nbytes3 = launch_bytes(base_bytes, prof3, vec3, n)
        out["preconditioners"] = {
            "cpr": {"value": v3, "ms_per_step": el3 / a.steps * 1e3, "p_iters": a.p_iters,
                    **{k: v for k, v in st3.items() if k != "nnzb"},
                    "roofline": roofline(prof3, nbytes3, wl.name), "kernel_classes": classes_of(prof3, nbytes3)},
            "cpr_over_bilu0_fp64": v3 / (v2 if mixed else value),
        }
        note(f"{wl.name}: BiCGSTAB")
        v4, el4, st4, prof4, vec4 = run_newton(wl, "fp64", a.inner, a.warmup, a.steps, krylov="bicgstab")
        nbytes4 = launch_bytes(base_bytes, prof4, vec4, n)
        out["krylov_methods"] = {
            "bicgstab": {"value": v4, "ms_per_step": el4 / a.steps * 1e3,
                         **{k: v for k, v in st4.items() if k != "nnzb"},
                         "roofline": roofline(prof4, nbytes4, wl.name),
                         "kernel_classes": classes_of(prof4, nbytes4)},
            "bicgstab_over_gmres_fp64": v4 / (v2 if mixed else value),
        }
    if not a.no_cpu_baseline:
        note("CPU baseline (the oracle)")
        out["cpu_baseline"] = cpu_baseline(wl, a.cpu_layers, a.cpu_workers)
    print(json.dumps(out), flush=True)
    # every context is destroyed by now; let the device drain before the
    # interpreter's own teardown
    import torch
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
