"""Benchmark: cells x Newton-iterations per second of the whole hot path
(assemble -> convergence check -> Gauss-Jordan decoupling -> BILU(0) ->
GMRES(30) to 1e-8 -> safeguarded update) on one MI355X.

A step is one Newton iteration that solves; when Newton has converged the
next timestep starts (the converged-check assembly is inside the timed
region, counted as no step).  Inputs are resident in HBM before timing.

    python bench.py [--steps K] [--warmup W] [--workload C3] [--precision fp64|mixed]
"""
from __future__ import annotations

import argparse
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
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--precision", default="fp64", choices=("fp64", "mixed"))
    ap.add_argument("--inner", type=int, default=6, help="FP32 inner iterations (mixed)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-layers", type=int, default=4, help="layers of the workload in the oracle sample")
    return ap.parse_args()


def algorithmic_bytes(n, nnzb, prec="fp64"):
    """Bytes each kernel class must move per launch (SURVEY-style counts:
    neighbour vector blocks assumed cache hits)."""
    b = 8 if prec == "fp64" else 4
    off = (nnzb - n) * 64 * b               # off-diagonal blocks of the decoupled matrix
    vec = n * 8 * 8                         # one FP64 block vector
    return {
        # y = A x: off-diagonal blocks + x + y
        "spmv": off + 2 * vec,
        # forward + backward sweep: all off-diagonal blocks once, D^-1 twice,
        # r read, v write, v read, z write
        "ilu_apply": off + 2 * n * 64 * 8 + 4 * vec,
        # u, u_old, porosity, 3 transmissibilities in; F and J out
        "assemble": 2 * vec + n * 8 * 4 + vec + nnzb * 64 * 8,
    }


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
                return info
            # failed step: restore and halve the step
            self.u.copy_(self.u_old)
            self.dt *= 0.5
            self.cuts += 1
            self.ni_in_step = 0
            if self.cuts > 40:
                raise RuntimeError(f"too many step cuts (status {st})")


def cpu_baseline(wl, layers):
    """The oracle, as it stands, on a bounded sample of the workload: one
    Newton iteration on its top `layers` layers."""
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
    t0 = time.perf_counter()
    st, u, info = m.newton_step(sub.u0, sub.u0, sub.dt)
    el = time.perf_counter() - t0
    return {"value": n / el, "unit": UNIT, "cores": 1, "kind": "oracle",
            "sample": f"one Newton iteration (assemble, decouple, BILU(0)-GMRES(30) to 1e-8, update) of the "
                      f"serial FP64 oracle on the top {layers} layers of {wl.name} ({n} cells), first step "
                      f"from the initial state; {info.iters_lin} GMRES iterations, {el:.1f} s",
            "status": int(st)}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (the hot path is single-GPU; see DESIGN.md for how it "
              f"would shard); got --gpus {a.gpus}", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1811_11992_amd import inputs as I
    from paper_1811_11992_amd import isc

    wl = I.make_workload(a.workload)
    mixed = a.precision == "mixed"
    ctx = isc.Context(wl, restart=30, inner_iters=a.inner if mixed else 0)
    lin = isc.solve_opts(restart=30, max_restarts=20, rtol=1e-8,
                         precision=isc.ISC_MIXED if mixed else isc.ISC_FP64, inner_iters=a.inner if mixed else 0)
    drv = Driver(ctx, wl, lin)
    for _ in range(a.warmup):
        drv.newton_iteration()
    torch.cuda.synchronize()
    ni0, lin0, inner0 = drv.ni, drv.lin_its, drv.inner_its
    isc.isc_profile(ctx, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        drv.newton_iteration()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = isc.isc_profile(ctx, 0)
    n = wl.ncell
    value = n * a.steps / el
    lin_per_ni = (drv.lin_its - lin0) / max(1, drv.ni - ni0)

    nbytes = algorithmic_bytes(n, ctx.nnzb)
    classes = {}
    for k, (ms, cnt) in prof.items():
        rec = {"ms": round(ms, 3), "launches": cnt}
        if k in nbytes and cnt > 0 and ms > 0:
            rec["GB_s"] = round(nbytes[k] * cnt / (ms * 1e-3) / 1e9, 1)
        classes[k] = rec
    dom = max((k for k in nbytes if prof[k][1] > 0), key=lambda k: prof[k][0])
    ms, cnt = prof[dom]
    achieved = nbytes[dom] / (ms / cnt * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": el / a.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if not mixed else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.nx}x{wl.ny}x{wl.nz} cells, "
                               + ("FP32 BILU(0) + inner SpMV in FP64 FGMRES(30)" if mixed
                                  else "FP64 BILU(0)-GMRES(30)") + " to 1e-8, Newton 1e-10",
                   "cells": n, "precision": a.precision, "newton_its_timed": a.steps,
                   "gmres_its_per_newton": round(lin_per_ni, 2), "timesteps_completed": drv.steps_done,
                   "step_cuts": drv.cuts},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_launch": nbytes[dom], "avg_launch_ms": round(ms / cnt, 4)},
        "kernel_classes": classes,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, a.cpu_layers)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
