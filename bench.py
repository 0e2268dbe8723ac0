"""Benchmark: target-point Stokes SL+DL evaluations per second on one MI355X.

A step is one full velocity evaluation of the two-drop workload (degree 32
drops 2.2 radii apart, viscosity ratios 1 and 5, linear equation of state):
geometry and force, region split, single layer (singular + pair sums),
Galerkin projection and GMRES on the second-kind equation (tolerance 1e-10),
velocity synthesis. Target-point evaluations = targets x (1 + operator
applications in the solve). Inputs are resident in device memory before the
timed region; the output is written to a device tensor.

Prints one JSON line (see the design doc for the roofline and baseline fields).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1707_02156_amd as B
    import workloads as W

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    wl = W.two_drops()
    with torch.cuda.stream(stream):
        ctx = B.Context(A_tilde=wl.A_tilde, U_tilde=wl.U_tilde, U_sing=wl.U_sing, U_geom=wl.U_geom,
                        gmres_tol=wl.gmres_tol, stream=stream.cuda_stream)
        ctx.set_drops([d.p for d in wl.drops], [d.xc for d in wl.drops], [d.lam for d in wl.drops])
        ctx.set_tension([d.gc for d in wl.drops], wl.eos, wl.E, wl.xs)
        out = torch.zeros(3 * ctx.ntargets(), dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            B.bim_eval_velocity(ctx.h, out)
        torch.cuda.synchronize()
        reps = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            reps.append(B.bim_eval_velocity(ctx.h, out))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    T = ctx.ntargets()
    evals = sum(T * (1 + r.n_matvec) for r in reps) / args.steps
    res = {
        "metric": "target-pt Stokes SL+DL evals/s",
        "value": evals / (ms * 1e-3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "two drops, p=32, gap 0.2, lambda (1,5), linear EOS, GMRES 1e-10, U=4",
                   "targets": T, "gmres_iterations": reps[-1].gmres_iterations,
                   "operator_applications": reps[-1].n_matvec},
    }
    print(json.dumps(res), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
