"""Times the linear-algebra kernels of one Newton iteration on a workload.

    python -m paper_1811_11992_amd.kernel_bench [--workload C3] [--reps 20] [--only linear|assemble]

Builds the decoupled Jacobian at the workload's initial state (assemble,
decouple, BILU(0) factor through the C-ABI), then times ``isc_bilu0_apply``,
``isc_spmv`` and the fused ``isc_bilu0_apply_spmv`` on a random right-hand
side (the public applies first form the L D^-1 blocks from their arguments),
and a plain device copy of one vector as the reference kernel for hardware
counters (a copy moves a known number of bytes).  Prints one JSON line.  Used
to take per-kernel traffic counters without the rest of the solver in the
trace.
"""
from __future__ import annotations

import argparse
import json
import time

import torch

from . import inputs as I
from . import isc


def assemble_only(wl, c, reps):
    """Times the property pass + face assembly alone (isc_assemble) at a state
    one Newton step away from the initial one, so that the reactions and the
    upstream choices are those of a burning front."""
    u0 = torch.tensor(wl.u0, dtype=torch.float64, device="cuda")
    u = u0.clone()
    st, info = c.isc_newton_step(u, u0, wl.dt)
    F, J = c.isc_assemble(u, u0, wl.dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        c.isc_assemble(u, u0, wl.dt, F, J)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    print(json.dumps({"workload": wl.name, "cells": c.n, "reps": reps, "assemble_ms": round(ms, 4),
                      "finite": bool(torch.isfinite(F).all())}), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--only", choices=("linear", "assemble", "factor"), default="linear",
                    help="time the linear-algebra kernels (default), the assembly alone, or the BILU(0) factor")
    a = ap.parse_args(argv)
    wl = I.make_workload(a.workload)
    c = isc.Context(wl)
    if a.only == "assemble":
        assemble_only(wl, c, a.reps)
        c.close()
        torch.cuda.synchronize()
        return
    u = torch.tensor(wl.u0, dtype=torch.float64, device="cuda")
    F, J = c.isc_assemble(u, u, wl.dt)
    c.isc_decouple(J, F)
    D = c.isc_bilu0(J)
    if a.only == "factor":
        # the factor of the first Newton iteration's decoupled matrix, again and again
        for _ in range(2):
            c.isc_bilu0(J, D)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.reps):
            c.isc_bilu0(J, D)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / a.reps * 1e3
        print(json.dumps({"workload": wl.name, "cells": c.n, "reps": a.reps, "bilu0_factor_ms": round(ms, 4),
                          "dinv_finite": bool(torch.isfinite(D).all()),
                          "dinv_sum": float(D.double().abs().sum())}), flush=True)
        c.close()
        torch.cuda.synchronize()
        return
    g = torch.Generator(device="cuda").manual_seed(1)
    r = torch.randn((c.n, 8), dtype=torch.float64, device="cuda", generator=g)
    z = torch.empty_like(r)
    y = torch.empty_like(r)
    for _ in range(3):
        c.isc_bilu0_apply(J, D, r, z)
    torch.cuda.synchronize()

    def timed(fn):
        t0 = time.perf_counter()
        for _ in range(a.reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / a.reps * 1e3

    t_apply = timed(lambda: c.isc_bilu0_apply(J, D, r, z))
    t_spmv = timed(lambda: c.isc_spmv(J, r, y))
    w = torch.empty_like(r)
    t_fused = timed(lambda: c.isc_bilu0_apply_spmv(J, D, r, z, w))
    t_copy = timed(lambda: y.copy_(r))
    vec_bytes = r.numel() * r.element_size()
    print(json.dumps({"workload": wl.name, "cells": c.n, "reps": a.reps, "bilu0_apply_ms": round(t_apply, 4),
                      "spmv_ms": round(t_spmv, 4), "apply_spmv_ms": round(t_fused, 4), "copy_ms": round(t_copy, 4),
                      "copy_bytes_each_way": vec_bytes, "apply_finite": bool(torch.isfinite(z).all())}), flush=True)
    c.close()
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
