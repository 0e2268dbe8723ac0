"""Benchmark: target-point Stokes SL+DL evaluations per second on one MI355X.

Workload (two drops, the configuration the metric is quoted on): degree-32
drops with N(0,1) 0.1 l^-3 perturbations, centres 2.2 apart (gap 0.2),
viscosity ratios 1 and 5, surfactant Gamma = 1 + 0.2 Y_2^0 with the linear
equation of state, Omega_1 threshold 5h with 4x upsampling, GMRES 1e-10.

A step is one full velocity evaluation: geometry and force, region split,
single layer (singular + pair sums; the stored singular double-layer rows are
built in the same pass), Galerkin projection, GMRES on the second-kind
equation, velocity synthesis. Target-point evaluations = targets x (1 + operator
applications in the solve). Inputs are resident in device memory before the
timed region; the output is written to a device tensor.

Extra fields: "roofline" for the kernel with the largest share of a step
(chosen from a short breakdown pass with every kernel timed; in the timed
region only that kernel is bracketed by HIP events on the library's stream,
since each event pair delays the next launch; algorithmic work from the
library's own counts), "kernels_ms_per_step" from the breakdown pass, and
"cpu_baseline": the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X peaks: FP64 vector (256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz), HBM3E
PEAK = {"alu": (78.6, "TFLOP/s"), "hbm": (8000.0, "GB/s")}
BOUND = {"sing_fused": "alu", "pair_sl": "alu", "pair_dl": "alu", "dl_apply": "hbm",
         "synthesis": "hbm", "analysis": "hbm", "sing_v1": "alu", "sing_rotate": "alu", "classify": "alu",
         "pipe_rotate": "alu", "pipe_legendre": "hbm", "pipe_fourier": "alu", "pipe_adjrot": "alu", "near": "alu",
         "fmm": "alu"}
KERNELS = list(BOUND)


WORKLOADS = {
    "two_drops": ("two drops p=32 (gap 0.2, lambda 1 and 5, linear EOS, U=4, A=5h), full velocity solve, "
                  "GMRES 1e-10"),
    "many_drops": ("64 drops p=16 (radii U[0.8,1.2], cube of side 12, gap >= 0.3, lambda in {1,2,5}, every pair "
                   "on the 2x grid), full velocity solve, GMRES 1e-10"),
    "deformed_drops": ("16 deformed drops p=48 (P2 spheroids D=0.3, pairs 0.1 apart, lambda 3, linear EOS, "
                       "U=4, A=5h), full velocity solve, GMRES 1e-10"),
    "single_drop": "single drop p=16 (lambda 1, uniform tension), velocity = single layer",
}

# HBM bytes per launch of a kernel from committed rocprofv3 counters
# (FETCH_SIZE x 2.0 and WRITE_SIZE x 1.0, the factors a plain copy of known
# size gives), valid while the kernel's source file is unchanged.
TRAFFIC = {("pipe_fourier", "two_drops"): ("profiles/pipe_fourier_two_drops_p32_counters.md",
                                           "paper_1707_02156_amd/csrc/kernels_pipe.hip")}


def workload(name):
    import workloads as W
    return getattr(W, name)()


def traffic(kernel, wname):
    """HBM bytes per launch recorded for this kernel and workload, or None if
    there is no record or the kernel source changed since it was taken."""
    import hashlib
    import re
    ent = TRAFFIC.get((kernel, wname))
    if not ent:
        return None
    prof, src = (os.path.join(ROOT, x) for x in ent)
    try:
        text = open(prof).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)\s+source_sha256:\s*([0-9a-f]{64})", text)
    if not m or m.group(2) != sha:
        return None
    return float(m.group(1))


def cpu_baseline(wl, budget_s=12.0):
    """The oracle on a bounded sample: single and double layer (singular rule
    plus pair sums) at batches of grid targets, alternating drops, until the
    time budget is used. Returns target-point evaluations per second."""
    import numpy as np

    import oracle
    o = oracle.Options(A_tilde=wl.A_tilde, U_tilde=wl.U_tilde, U_sing=wl.U_sing, U_geom=wl.U_geom,
                       eos=wl.eos, E=wl.E, xs=wl.xs, sigma0=wl.sigma0)
    s = oracle.System([oracle.Drop(d.p, d.xc, d.lam, d.gc) for d in wl.drops], o)
    f = [s.force(i) for i in range(len(wl.drops))]
    for i in range(min(len(wl.drops), 64)):     # setup outside the clock: regions and tables
        s.layer(i, f, 0, targets=np.arange(2))
    rng = np.random.default_rng(0)
    evals, t_used, batches = 0, 0.0, 0
    while t_used < budget_s and batches < 64:
        i = batches % len(wl.drops)
        tg = np.sort(rng.choice(oracle.npts(wl.drops[i].p), 64, replace=False))
        t0 = time.perf_counter()
        s.layer(i, f, 0, targets=tg)            # single layer at the sample
        s.layer(i, f, 1, targets=tg)            # double layer at the sample
        t_used += time.perf_counter() - t0
        evals += 2 * len(tg)
        batches += 1
    return {"value": evals / t_used, "unit": "evals/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{evals} target-point evaluations (single and double layer, {batches} batches of 64 grid "
                      f"targets alternating drops) in {t_used:.1f} s"}


def serve(args):
    """Serving stream (2048 systems of 1-8 drops, p in {8, 16, 24, 32},
    lambda in {1, 2, 5}, Poisson arrivals): one-at-a-time capacity of a plain
    context, then the stream at rate_factor x that capacity through a 1-slot
    server (one request at a time) and through the slotted server (continuous
    admission, overlapping requests); p50/p99 arrival-to-finish latency and
    throughput of each."""
    import threading

    import numpy as np
    import torch

    import paper_1707_02156_amd as B
    import workloads as W

    torch.cuda.set_device(0)
    reqs = W.serving_requests(n=args.requests)
    opts = dict(fmm_order=args.fmm_order, fmm_eps=args.fmm_eps,
                precision=B.BIM_PREC_MIXED if args.precision == "mixed" else B.BIM_PREC_FP64)
    ctx = B.Context(**opts)

    def alone(r):
        ctx.set_drops([d.p for d in r.drops], [d.xc for d in r.drops], [d.lam for d in r.drops])
        ctx.set_tension(None, 0, sigma0=1.0)
        return ctx.eval_velocity()[1]

    for r in reqs[:8]:
        alone(r)
    sample = reqs[: min(len(reqs), args.capacity_sample)]
    t0 = time.perf_counter()
    for r in sample:
        alone(r)
    mean_s = (time.perf_counter() - t0) / len(sample)
    ctx.close()
    capacity = 1.0 / mean_s

    def stream(slots, rate, batch=1):
        srv = B.Server(slots=slots, max_batch=batch, **opts)
        for r in reqs[:8]:   # warm the contexts' tables
            srv.wait(srv.submit([d.p for d in r.drops], [d.xc for d in r.drops], [d.lam for d in r.drops]))
        ids, lat, evals = [], [], [0]
        done = threading.Event()

        def collect():
            k = 0
            while k < len(reqs):
                if k >= len(ids):
                    time.sleep(0.0005)
                    continue
                res = srv.wait(ids[k])
                u, rep, t = res
                lat.append(t[2])
                evals[0] += rep.n_targets * (1 + rep.n_matvec)
                k += 1
            done.set()

        th = threading.Thread(target=collect)
        th.start()
        start = time.perf_counter()
        for r in reqs:
            delay = start + r.arrival / rate - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            ids.append(srv.submit([d.p for d in r.drops], [d.xc for d in r.drops], [d.lam for d in r.drops]))
        done.wait()
        th.join()
        span = time.perf_counter() - start
        srv.close()
        lat = np.array(lat)
        return {"slots": slots, "max_batch": batch, "rate_req_s": rate, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "throughput_req_s": len(reqs) / span,
                "evals_per_s": evals[0] / span}

    rate = args.rate_factor * capacity
    runs = [stream(1, rate), stream(args.slots, rate), stream(args.slots, rate, args.max_batch)]
    for f in (1.5, 2.0, 4.0):
        runs.append(stream(args.slots, f * capacity))
        runs.append(stream(args.slots, f * capacity, args.max_batch))
    res = {"metric": "p50/p99 solve latency and throughput of the serving stream", "requests": len(reqs),
           "capacity_one_at_a_time_req_s": capacity, "mean_service_ms": mean_s * 1e3,
           "rate_factor": args.rate_factor, "runs": runs,
           "dtype": "f64" if args.precision == "fp64" else "f64 (pair sums f32)", "data": "synthetic",
           "config": {"workload": "serving stream: 1-8 drops, p in {8,16,24,32}, lambda in {1,2,5}, gap >= 0.2, "
                                  "Poisson arrivals"}}
    print(json.dumps(res), flush=True)


def kernel_frac(name, d):
    """Achieved fraction of the kernel's roofline (algorithmic work / event time)."""
    bound = BOUND[name]
    peak, _ = PEAK[bound]
    sec = d["ms"] * 1e-3
    if bound == "hbm":
        return d["bytes"] / sec / 1e9 / peak
    return d["flops"] / sec / 1e12 / peak


def time_loop(args):
    """Coupled drop / surfactant time stepping (bim_time_step) of the two-drop
    p=32 workload in a shear flow with its surfactant: adaptive steps from
    dt0; reports time steps per second, target-point evaluations per second
    (both velocity solves of every step), acceptance, dt, and the drift of the
    total surfactant over the run."""
    import numpy as np
    import torch

    import paper_1707_02156_amd as B

    torch.cuda.set_device(0)
    wl = workload("two_drops")
    shear = np.zeros((3, 3))
    shear[0, 1] = args.shear
    ctx = B.Context(A_tilde=wl.A_tilde, U_tilde=wl.U_tilde, U_sing=wl.U_sing, U_geom=wl.U_geom,
                    gmres_tol=wl.gmres_tol, fmm_order=args.fmm_order, fmm_eps=args.fmm_eps,
                    precision=B.BIM_PREC_MIXED if args.precision == "mixed" else B.BIM_PREC_FP64)
    ctx.set_drops([d.p for d in wl.drops], [d.xc for d in wl.drops], [d.lam for d in wl.drops])
    ctx.set_tension([d.gc for d in wl.drops], wl.eos, wl.E, wl.xs)
    B.bim_set_farfield(ctx.h, np.zeros(3), shear)
    dt = args.dt0
    for _ in range(args.warmup):                  # warm-up: steps with tol <= 0 are always accepted
        ctx.time_step(dt, Pe=args.pe, tol=0.0)
    T = ctx.ntargets()
    reps = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rreps = []
    for _ in range(args.steps):
        r = ctx.time_step(dt, Pe=args.pe, tol=args.tol)
        reps.append(r)
        if r["accepted"] and args.rep_imax > 0:   # Algorithm 1: reparametrize after an accepted step
            rreps.append(ctx.reparametrize(U_rep=2, P_cut=args.rep_pcut, eps=args.rep_eps, imax=args.rep_imax))
        dt = min(r["dt_next"], args.dt_max)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.close()
    ms = (t1 - t0) * 1e3 / args.steps
    evals = sum(T * (2 + r["gmres_velocity"][0] + r["gmres_velocity"][1]) for r in reps) / args.steps
    acc = [r for r in reps if r["accepted"]]
    res = {
        "metric": "coupled drop/surfactant time steps/s",
        "value": 1e3 / ms,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "dtype": "f64" if args.precision == "fp64" else "f64 (pair sums f32)",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["two_drops"] + f"; shear rate {args.shear}, Pe {args.pe}, "
                   f"adaptive dt (tol {args.tol}, dt0 {args.dt0}, dt_max {args.dt_max})", "targets": T},
        "evals_per_s": evals / (ms * 1e-3),
        "accepted": len(acc),
        "dt_last": dt,
        "gmres_velocity_mean": float(np.mean([sum(r["gmres_velocity"]) / 2 for r in reps])),
        "gmres_imex_mean": float(np.mean([r["gmres_imex"] for r in reps])),
        "err_surf_max_accepted": max((r["err_surf"] for r in acc), default=0.0),
        "mass_drift": (acc[-1]["mass1"] / acc[0]["mass0"] - 1.0) if acc else 0.0,
    }
    if rreps:
        res["reparametrization"] = {"calls": len(rreps), "ms_mean": float(np.mean([r["ms_total"] for r in rreps])),
                                    "moves_mean": float(np.mean([r["moves"] for r in rreps])),
                                    "U_rep": 2, "P_cut": args.rep_pcut, "eps": args.rep_eps, "imax": args.rep_imax}
        res["config"]["workload"] += f"; reparametrization after accepted steps (imax {args.rep_imax})"
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--singular-path", type=int, default=0)
    ap.add_argument("--workload", default="two_drops", choices=list(WORKLOADS),
                    help="two_drops is the configuration the metric is quoted on; the others are reported in "
                         "the design notes")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the workload, copy a buffer of this size three times (a plain copy of known "
                         "size against which the HBM byte counters are scaled)")
    ap.add_argument("--serve", action="store_true", help="run the serving stream instead of the step benchmark")
    ap.add_argument("--requests", type=int, default=2048)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--rate-factor", type=float, default=0.8)
    ap.add_argument("--capacity-sample", type=int, default=128)
    ap.add_argument("--max-batch", type=int, default=16)
    ap.add_argument("--time-loop", action="store_true", help="run the coupled drop / surfactant time stepping")
    ap.add_argument("--pe", type=float, default=200.0)
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--dt0", type=float, default=0.05)
    ap.add_argument("--dt-max", type=float, default=0.2)
    ap.add_argument("--shear", type=float, default=0.2)
    ap.add_argument("--rep-imax", type=int, default=0, help="time loop: reparametrize after accepted steps (0: off)")
    ap.add_argument("--fmm-order", type=int, default=0,
                    help="fast summation of far drop pairs: multipole order P (0: every pair summed directly)")
    ap.add_argument("--fmm-eps", type=float, default=1e-10, help="truncation bound rho^(P+1) of a far pair")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="mixed: the direct pair sums in FP32 arithmetic, the rest in FP64")
    ap.add_argument("--rep-pcut", type=float, default=1e-3)
    ap.add_argument("--rep-eps", type=float, default=1e-6)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; multi-GPU runs are not part of it (use --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    if args.serve:
        serve(args)
        return
    if args.time_loop:
        time_loop(args)
        return

    import torch

    import paper_1707_02156_amd as B

    torch.cuda.set_device(0)
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    wl = workload(args.workload)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = B.Context(A_tilde=wl.A_tilde, U_tilde=wl.U_tilde, U_sing=wl.U_sing, U_geom=wl.U_geom,
                        gmres_tol=wl.gmres_tol, singular_path=args.singular_path, stream=stream.cuda_stream,
                        fmm_order=args.fmm_order, fmm_eps=args.fmm_eps,
                        precision=B.BIM_PREC_MIXED if args.precision == "mixed" else B.BIM_PREC_FP64)
        ctx.set_drops([d.p for d in wl.drops], [d.xc for d in wl.drops], [d.lam for d in wl.drops])
        if wl.eos != 0:
            ctx.set_tension([d.gc for d in wl.drops], wl.eos, wl.E, wl.xs)
        else:
            ctx.set_tension(None, 0, sigma0=wl.sigma0)
        out = torch.zeros(3 * ctx.ntargets(), dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            B.bim_eval_velocity(ctx.h, out)
        torch.cuda.synchronize()
        # kernel breakdown: a few untimed steps with every kernel bracketed by events
        nprof = max(1, min(3, args.steps))
        B.bim_profile(ctx.h, 1)
        for _ in range(nprof):
            B.bim_eval_velocity(ctx.h, out)
        brk = {k: B.bim_profile_query(ctx.h, k) for k in KERNELS}
        B.bim_profile(ctx.h, 0)
        dom = max(brk, key=lambda k: brk[k]["ms"])
        # timed region: events only around the dominant kernel
        B.bim_profile_select(ctx.h, [dom])
        B.bim_profile(ctx.h, 1)
        reps = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            reps.append(B.bim_eval_velocity(ctx.h, out))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        d = B.bim_profile_query(ctx.h, dom)
        B.bim_profile(ctx.h, 0)
        B.bim_profile_select(ctx.h, None)
    ms = (t1 - t0) * 1e3 / args.steps
    T = ctx.ntargets()
    evals = sum(T * (1 + r.n_matvec) for r in reps) / args.steps
    bound = BOUND[dom]
    peak, unit = PEAK[bound]
    per_launch_s = d["ms"] * 1e-3 / max(d["launches"], 1)
    if bound == "hbm":
        achieved = d["bytes"] / max(d["launches"], 1) / per_launch_s / 1e9
    else:
        achieved = d["flops"] / max(d["launches"], 1) / per_launch_s / 1e12
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
        "dtype": "f64" if args.precision == "fp64" else "f64 (pair sums f32)",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload],
                   "targets": T, "gmres_iterations": reps[-1].gmres_iterations,
                   "operator_applications": reps[-1].n_matvec},
        "roofline": {"kernel": dom, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                     "frac": achieved / peak, "traffic": traffic(dom, args.workload),
                     "avg_launch_us": per_launch_s * 1e6, "launches": d["launches"],
                     "share_of_step": d["ms"] / (ms * args.steps)},
        "kernels_ms_per_step": {k: round(v["ms"] / nprof, 4) for k, v in brk.items() if v["launches"]},
        "kernels_roofline_frac": {k: round(kernel_frac(k, v), 4) for k, v in brk.items() if v["ms"] > 0},
    }
    if args.fmm_order != 0:
        res["config"]["fast_summation"] = {"order": reps[-1].fmm_order, "eps": args.fmm_eps,
                                           "far_pairs": reps[-1].n_fmm_pairs,
                                           "chosen_by_timing": args.fmm_order < 0}
    ctx.close()
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
