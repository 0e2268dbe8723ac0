"""Benchmark: target-point Stokes SL+DL evaluations per second on one MI355X.

Default workload (the largest single-GPU configuration): 16 strongly deformed
drops of degree 48 (P2 spheroids of Taylor deformation 0.3 with N(0,1) 0.05
l^-3 noise, random orientations), surfactant of degree 48 with the linear
equation of state, viscosity ratio 3, eight close pairs 0.1 apart on a
lattice of spacing 8, Omega_1 threshold 5h with 4x upsampling, GMRES 1e-10.

A step is one full velocity evaluation in FP64 (the plain form: every pair
summed directly): geometry and force, region split, single layer (singular +
pair sums; the stored singular double-layer rows are built in the same pass),
Galerkin projection, GMRES on the second-kind equation, velocity synthesis.
Target-point evaluations = targets x (1 + operator applications in the
solve). Inputs are resident in device memory before the timed region; the
output is written to a device tensor.

Extra fields:
- "roofline" for the kernel with the largest share of a step (chosen from a
  short breakdown pass with every kernel timed; in the timed region only that
  kernel is bracketed by HIP events on the library's stream, since each event
  pair delays the next launch; algorithmic work from the library's counts);
- "vs_baseline": the fastest other form of the same evaluation whose output
  stays within the FP64 parity bar (1e-10 per drop and component) of the
  plain form, divided by the plain form's rate; "forms" lists every form
  measured (fast summation in FP64, FP32 far field, both) with its rate and
  its largest deviation from the plain form;
- "latency": p50/p99 arrival-to-finish latency of a bounded serving stream
  (systems of 1-8 drops, p in {8, 16, 24, 32}, Poisson arrivals at 0.8x the
  one-at-a-time capacity; FP32 far field, FP64 singular steps) through the
  continuous-batching server and one request at a time;
- "kernels_ms_per_step" from the breakdown pass;
- "cpu_baseline": the CPU oracle timed on a bounded sample of the workload.
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
BOUND = {"sing_fused": "alu", "pair_sl": "alu", "pair_dl": "alu",
         "pair_gather": "hbm", "pair_pack": "hbm", "dl_apply": "hbm",
         "synthesis": "hbm", "analysis": "hbm", "sing_v1": "alu", "sing_rotate": "alu", "classify": "alu",
         "pipe_rotate": "alu", "pipe_legendre": "hbm", "pipe_fourier": "alu", "pipe_adjrot": "alu", "near": "alu",
         "fmm": "alu"}
KERNELS = list(BOUND)


WORKLOADS = {
    "deformed_drops": ("16 deformed drops p=48 (P2 spheroids D=0.3, pairs 0.1 apart, lambda 3, linear EOS, "
                       "U=4, A=5h), full velocity solve, GMRES 1e-10"),
    "two_drops": ("two drops p=32 (gap 0.2, lambda 1 and 5, linear EOS, U=4, A=5h), full velocity solve, "
                  "GMRES 1e-10"),
    "many_drops": ("64 drops p=16 (radii U[0.8,1.2], cube of side 12, gap >= 0.3, lambda in {1,2,5}, every pair "
                   "on the 2x grid), full velocity solve, GMRES 1e-10"),
    "single_drop": "single drop p=16 (lambda 1, uniform tension), velocity = single layer",
}

# HBM bytes per launch of a kernel from committed rocprofv3 counters
# (FETCH_SIZE x 2.0 and WRITE_SIZE x 1.0, the factors a plain copy of known
# size gives), valid while the kernel's source file is unchanged.
TRAFFIC = {("pair_dl", "deformed_drops"): ("profiles/pair_dl_deformed_drops_p48_counters.md",
                                            "paper_1707_02156_amd/csrc/kernels.hip")}


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
    nd = min(len(wl.drops), 2)                  # the sample alternates between the first two drops
    for i in range(nd):                         # setup outside the clock: regions and tables
        s.layer(i, f, 0, targets=np.arange(2))
    rng = np.random.default_rng(0)
    evals, t_used, batches = 0, 0.0, 0
    while t_used < budget_s and batches < 64:
        i = batches % nd
        tg = np.sort(rng.choice(oracle.npts(wl.drops[i].p), 64, replace=False))
        t0 = time.perf_counter()
        s.layer(i, f, 0, targets=tg)            # single layer at the sample
        s.layer(i, f, 1, targets=tg)            # double layer at the sample
        t_used += time.perf_counter() - t0
        evals += 2 * len(tg)
        batches += 1
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": evals / t_used, "unit": "evals/s", "cores": oracle.num_threads(), "kind": "oracle",
            "cpu": cpu,
            "sample": f"{evals} target-point evaluations (single and double layer, {batches} batches of 64 grid "
                      f"targets alternating between the first two drops) in {t_used:.1f} s"}


def serving_opts(B, args):
    return dict(fmm_order=args.fmm_order, fmm_eps=args.fmm_eps,
                precision=B.BIM_PREC_MIXED if args.precision == "mixed" else B.BIM_PREC_FP64)


def capacity(B, reqs, opts, nsample):
    """One-at-a-time capacity (requests/s) of a plain context with the
    server's work-shape options (no timing of shapes) over the first nsample
    requests (after 8 warm-up requests)."""
    ctx = B.Context(pair_tune=0, xform_path=1, **opts)

    def alone(r):
        ctx.set_drops([d.p for d in r.drops], [d.xc for d in r.drops], [d.lam for d in r.drops])
        ctx.set_tension(None, 0, sigma0=1.0)
        return ctx.eval_velocity()[1]

    for r in reqs[:8]:
        alone(r)
    sample = reqs[: min(len(reqs), nsample)]
    t0 = time.perf_counter()
    for r in sample:
        alone(r)
    mean_s = (time.perf_counter() - t0) / len(sample)
    ctx.close()
    return 1.0 / mean_s, mean_s


def stream(B, reqs, opts, slots, rate, batch=1, max_queue=0):
    """The requests through a server of `slots` slots (batches of up to
    `batch`, at most `max_queue` waiting, 0: no limit), submitted at their
    Poisson arrival times scaled to `rate`; p50/p99 arrival-to-finish latency
    of the served requests, throughput, and the fraction refused."""
    import threading

    import numpy as np
    srv = B.Server(slots=slots, max_batch=batch, max_queue=max_queue, **opts)
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
            if ids[k] is not None:   # None: refused at submission
                u, rep, t = srv.wait(ids[k])
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
        try:
            ids.append(srv.submit([d.p for d in r.drops], [d.xc for d in r.drops], [d.lam for d in r.drops]))
        except B.BimError as e:
            if e.status != B.BIM_EBUSY:
                raise
            ids.append(None)
    done.wait()
    th.join()
    span = time.perf_counter() - start
    srv.close()
    lat = np.array(lat)
    return {"slots": slots, "max_batch": batch, "rate_req_s": rate, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "throughput_req_s": len(lat) / span,
            "evals_per_s": evals[0] / span, "refused": sum(i is None for i in ids) / len(ids)}


def serve(args):
    """Serving stream (systems of 1-8 drops, p in {8, 16, 24, 32}, lambda in
    {1, 2, 5}, Poisson arrivals): one-at-a-time capacity of a plain context,
    then the stream at rate_factor x that capacity through a 1-slot server
    (one request at a time) and through the slotted server (continuous
    admission, overlapping requests), and at 1.5, 2 and 4 x the capacity;
    p50/p99 arrival-to-finish latency and throughput of each."""
    import torch

    import paper_1707_02156_amd as B
    import workloads as W

    torch.cuda.set_device(0)
    reqs = W.serving_requests(n=args.requests)
    opts = serving_opts(B, args)
    cap, mean_s = capacity(B, reqs, opts, args.capacity_sample)
    rate = args.rate_factor * cap
    runs = [stream(B, reqs, opts, 1, rate), stream(B, reqs, opts, args.slots, rate),
            stream(B, reqs, opts, args.slots, rate, args.max_batch)]
    for f in (1.5, 2.0, 4.0):
        runs.append(stream(B, reqs, opts, args.slots, f * cap))
        runs.append(stream(B, reqs, opts, args.slots, f * cap, args.max_batch))
    res = {"metric": "p50/p99 solve latency and throughput of the serving stream", "requests": len(reqs),
           "capacity_one_at_a_time_req_s": cap, "mean_service_ms": mean_s * 1e3,
           "rate_factor": args.rate_factor, "runs": runs,
           "dtype": "f64" if args.precision == "fp64" else "f64 (pair sums f32)", "data": "synthetic",
           "config": {"workload": "serving stream: 1-8 drops, p in {8,16,24,32}, lambda in {1,2,5}, gap >= 0.2, "
                                  "Poisson arrivals"}}
    print(json.dumps(res), flush=True)


def latency(args):
    """Bounded serving stream for the headline line: args.latency_requests
    systems of the serving stream, FP32 far field and FP64 singular steps
    (as that workload specifies), at 0.8x the one-at-a-time capacity through
    the continuous-batching server (args.slots slots) and one at a time."""
    import paper_1707_02156_amd as B
    import workloads as W
    reqs = W.serving_requests(n=args.latency_requests)
    opts = dict(precision=B.BIM_PREC_MIXED)
    cap, mean_s = capacity(B, reqs, opts, min(64, len(reqs)))
    rate = 0.8 * cap
    served = stream(B, reqs, opts, args.slots, rate)
    single = stream(B, reqs, opts, 1, rate)
    over = {k: stream(B, reqs, opts, s_, 1.5 * cap) for k, s_ in (("served", args.slots), ("one_at_a_time", 1))}
    # overload: 3x the capacity, with and without a bound on the waiting requests
    shed = {k: stream(B, reqs, opts, args.slots, 3.0 * cap, max_queue=mq)
            for k, mq in ((f"max_queue_{2 * args.slots}", 2 * args.slots), ("unbounded", 0))}
    return {"p50_ms": served["p50_ms"], "p99_ms": served["p99_ms"],
            "throughput_req_s": served["throughput_req_s"], "evals_per_s": served["evals_per_s"],
            "one_at_a_time": {"p50_ms": single["p50_ms"], "p99_ms": single["p99_ms"],
                              "throughput_req_s": single["throughput_req_s"]},
            "at_1.5x_capacity": {k: {"p50_ms": v["p50_ms"], "p99_ms": v["p99_ms"],
                                     "throughput_req_s": v["throughput_req_s"]} for k, v in over.items()},
            "at_3x_capacity": {k: {"p50_ms": v["p50_ms"], "p99_ms": v["p99_ms"],
                                   "throughput_req_s": v["throughput_req_s"], "refused": v["refused"]}
                               for k, v in shed.items()},
            "requests": len(reqs), "slots": args.slots, "rate_req_s": rate, "capacity_one_at_a_time_req_s": cap,
            "workload": "serving stream: systems of 1-8 drops, p in {8,16,24,32}, lambda in {1,2,5}, gap >= 0.2, "
                        "Poisson arrivals at 0.8x the one-at-a-time capacity; FP32 far field, FP64 singular "
                        "steps and GMRES"}


def kernel_peak(name, mixed):
    """(bound, peak, unit) of a kernel group: FP32 vector peak for the pair
    sums of the mixed form, else FP64 vector (ALU) or HBM."""
    bound = BOUND[name]
    if bound == "alu" and mixed and name.startswith("pair_") and name not in ("pair_gather", "pair_pack"):
        return bound, 157.3, "TFLOP/s"
    peak, unit = PEAK[bound]
    return bound, peak, unit


def kernel_frac(name, d, mixed=False):
    """Achieved fraction of the kernel's roofline (algorithmic work / event time)."""
    bound, peak, _ = kernel_peak(name, mixed)
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


def make_ctx(B, wl, stream, **opts):
    ctx = B.Context(A_tilde=wl.A_tilde, U_tilde=wl.U_tilde, U_sing=wl.U_sing, U_geom=wl.U_geom,
                    gmres_tol=wl.gmres_tol, stream=stream.cuda_stream, **opts)
    ctx.set_drops([d.p for d in wl.drops], [d.xc for d in wl.drops], [d.lam for d in wl.drops])
    if wl.eos != 0:
        ctx.set_tension([d.gc for d in wl.drops], wl.eos, wl.E, wl.xs)
    else:
        ctx.set_tension(None, 0, sigma0=wl.sigma0)
    return ctx


def max_rel_dev(a, b, ps):
    """Largest over drops and components of ||a - b||_inf / ||b||_inf on the
    drop's grid (grid outputs [3][T])."""
    import numpy as np
    a = a.reshape(3, -1)
    b = b.reshape(3, -1)
    out, o = 0.0, 0
    for p in ps:
        n = 2 * p * (p + 1)
        for c in range(3):
            den = float(np.abs(b[c, o:o + n]).max())
            if den > 0.0:
                out = max(out, float(np.abs(a[c, o:o + n] - b[c, o:o + n]).max()) / den)
        o += n
    return out


def timed_form(B, wl, args, steps, warmup, **opts):
    """Velocity evaluations of one form: (ms per step, evals/s, output on the
    host, last report)."""
    import torch
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = make_ctx(B, wl, stream, **opts)
        out = torch.zeros(3 * ctx.ntargets(), dtype=torch.float64, device="cuda")
        for _ in range(warmup):
            B.bim_eval_velocity(ctx.h, out)
        torch.cuda.synchronize()
        reps = []
        t0 = time.perf_counter()
        for _ in range(steps):
            reps.append(B.bim_eval_velocity(ctx.h, out))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        T = ctx.ntargets()
        ctx.close()
    ms = (t1 - t0) * 1e3 / steps
    evals = sum(T * (1 + r.n_matvec) for r in reps) / steps
    return ms, evals / (ms * 1e-3), out.cpu().numpy(), reps[-1]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the other forms (vs_baseline stays null)")
    ap.add_argument("--no-latency", action="store_true", help="skip the bounded serving stream")
    ap.add_argument("--latency-requests", type=int, default=256)
    ap.add_argument("--form-steps", type=int, default=5)
    ap.add_argument("--singular-path", type=int, default=0)
    ap.add_argument("--workload", default="deformed_drops", choices=list(WORKLOADS),
                    help="deformed_drops (16 drops p=48) is the headline; the others are reported in the design "
                         "notes")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the workload, copy a buffer of this size three times (a plain copy of known "
                         "size against which the HBM byte counters are scaled)")
    ap.add_argument("--serve", action="store_true", help="run the serving stream instead of the step benchmark")
    ap.add_argument("--requests", type=int, default=2048)
    ap.add_argument("--slots", type=int, default=3)
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
    mixed = args.precision == "mixed"
    opts = dict(singular_path=args.singular_path, fmm_order=args.fmm_order, fmm_eps=args.fmm_eps,
                precision=B.BIM_PREC_MIXED if mixed else B.BIM_PREC_FP64)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = make_ctx(B, wl, stream, **opts)
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
        ps = list(ctx.ps)
        T = ctx.ntargets()
        ctx.close()
    u_plain = out.cpu().numpy()
    ms = (t1 - t0) * 1e3 / args.steps
    evals = sum(T * (1 + r.n_matvec) for r in reps) / args.steps
    value = evals / (ms * 1e-3)
    bound, peak, unit = kernel_peak(dom, mixed)
    per_launch_s = d["ms"] * 1e-3 / max(d["launches"], 1)
    if bound == "hbm":
        achieved = d["bytes"] / max(d["launches"], 1) / per_launch_s / 1e9
    else:
        achieved = d["flops"] / max(d["launches"], 1) / per_launch_s / 1e12
    res = {
        "metric": "target-pt Stokes SL+DL evals/s",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if not mixed else "f64 (pair sums f32)",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload],
                   "targets": T, "gmres_iterations": reps[-1].gmres_iterations,
                   "operator_applications": reps[-1].n_matvec,
                   "pair_shape": {"targets_per_lane": reps[-1].pair_targets_per_lane,
                                  "sources_per_item": reps[-1].pair_sources_per_item,
                                  "chosen_by_timing": True},
                   "transforms": {"synthesis": "matrix cores" if reps[-1].xform_matrix_cores & 1 else "scalar",
                                  "analysis": "matrix cores" if reps[-1].xform_matrix_cores & 2 else "scalar",
                                  "chosen_by_timing": True}},
        "roofline": {"kernel": dom, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                     "frac": achieved / peak, "traffic": traffic(dom, args.workload),
                     "avg_launch_us": per_launch_s * 1e6, "launches": d["launches"],
                     "share_of_step": d["ms"] / (ms * args.steps)},
        "kernels_ms_per_step": {k: round(v["ms"] / nprof, 4) for k, v in brk.items() if v["launches"]},
        "kernels_roofline_frac": {k: round(kernel_frac(k, v, mixed), 4) for k, v in brk.items() if v["ms"] > 0},
    }
    if args.fmm_order != 0:
        res["config"]["fast_summation"] = {"order": reps[-1].fmm_order, "eps": args.fmm_eps,
                                           "far_pairs": reps[-1].n_fmm_pairs,
                                           "chosen_by_timing": args.fmm_order < 0}
    plain = not mixed and args.fmm_order == 0 and args.singular_path == 0
    if plain and not args.no_forms:
        # the same evaluation in the library's other forms, against the plain form's output
        forms = {}
        cand = [("pair_shape_by_rule", dict(pair_tune=0)),
                ("fast_summation_fp64", dict(fmm_order=-1, fmm_eps=1e-12)),
                ("fp32_far_field", dict(precision=B.BIM_PREC_MIXED)),
                ("fp32_far_field_fast_summation", dict(precision=B.BIM_PREC_MIXED, fmm_order=-1, fmm_eps=1e-8))]
        for name, o in cand:
            fms, fval, fu, frep = timed_form(B, wl, args, args.form_steps, 2, **o)
            forms[name] = {"ms_per_step": fms, "evals_per_s": fval, "ratio_to_plain": fval / value,
                           "max_rel_dev_from_plain": max_rel_dev(fu, u_plain, ps),
                           "gmres_iterations": frep.gmres_iterations, "fmm_order": frep.fmm_order,
                           "far_pairs": frep.n_fmm_pairs, "options": {k: v for k, v in o.items()}}
        eq = {k: v for k, v in forms.items() if v["max_rel_dev_from_plain"] <= 1e-10}
        if eq:
            best = max(eq, key=lambda k: eq[k]["evals_per_s"])
            res["vs_baseline"] = eq[best]["ratio_to_plain"]
            res["vs_baseline_form"] = {"form": best, "baseline": "plain FP64 GPU form (every pair summed "
                                       "directly), this line's value", "accuracy": "largest per-drop, "
                                       "per-component relative deviation from the plain form <= 1e-10 (FP64 "
                                       "parity bar)"}
        res["forms"] = forms
    if not args.no_latency:
        res["latency"] = latency(args)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
