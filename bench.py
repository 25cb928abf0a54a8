"""Benchmark of one IMEX-RK step of resistive GRMHD on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (value): the 3-D magnetised polytropic star in a static conformally
flat metric (Cowling), 128^3 cells on [-12, 12]^3, PPM + HLL + upwind CT +
IMEX-SSP3(4,3,3), FP64, seeded synthetic initial data (TOV equilibrium built
by the generator, poloidal field from a vector potential).  A step is one
full pass of the hot path (all IMEX stages and the final recovery).
value = interior cells x timed steps / seconds (zone-cycles/s), inputs
resident in HBM.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector


def time_steps(run, dt, steps, torch):
    s = run.stream
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        run.step(dt)
    e1.record(s)
    e1.synchronize()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def kernel_roofline(run, dt, steps, grmhd, torch):
    """replay of the timed steps with every kernel class bracketed by HIP
    events on the run's stream; roofline of the class with the largest time"""
    n_cls = 0
    while grmhd.gr_kernel_class_name(n_cls):
        n_cls += 1
    grmhd.gr_timing_start((1 << n_cls) - 1)
    torch.cuda.synchronize()
    for _ in range(steps):
        run.step(dt)
    torch.cuda.synchronize()
    per = {}
    for c in range(n_cls):
        ms, n, by = grmhd.gr_timing_read(c)
        if n:
            per[grmhd.gr_kernel_class_name(c)] = (ms, n, by)
    grmhd.gr_timing_start(0)
    name = max(per, key=lambda k: per[k][0])
    ms, n, by = per[name]
    achieved = by / (ms * 1e-3) / 1e9
    return name, {
        "bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
        "avg_launch_us": round(ms * 1e3 / n, 2), "launches": n, "alg_bytes_per_launch": by / n,
    }, {k: {"ms_per_step": round(v[0] / steps, 4), "launches_per_step": v[1] / steps,
            "alg_GBps": round(v[2] / (v[0] * 1e-3) / 1e9, 1)} for k, v in per.items()}


def cpu_baseline(setup_fn):
    import oracle
    s = setup_fn()
    st = oracle.OracleState(s)
    dt = st.dt()
    t0 = time.time()
    st.step(dt)
    el = time.time() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(s.ncells / el, 1), "unit": "zone-cycles/s", "cores": cores, "kind": "oracle",
            "sample": "one full IMEX-SSP3 step of the same %dx%dx%d star (%.1f s, OpenMP threads=%d)" % (
                s.n[0], s.n[1], s.n[2], el, cores)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=128, help="cells per direction of the star workload")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extra", action="store_true", help="star workload only (no 2-D point, no roofline replay)")
    ap.add_argument("--copy-ref", action="store_true",
                    help="end with a plain 256 MiB device copy, the reference kernel for scaling HBM counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build measures one MI355X only; runs on more than one GPU are not supported "
              "(independent runs shard by whole runs, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    from paper_2110_03732_amd import grmhd
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)

    def star():
        return W.tov_star(args.n)

    s = star()
    run = grmhd.Run(s, device="cuda:0")
    dt = run.dt()
    for _ in range(args.warmup):
        run.step(dt)
    ms = time_steps(run, dt, args.steps, torch)
    ms_per_step = ms / args.steps
    value = s.ncells * args.steps / (ms * 1e-3)
    fails = run.fail_count()
    div = run.divB()
    extra = {"recovery_failures": int(fails), "divB_linf": float(div[2])}
    roof = None
    if not args.no_extra:
        kname, roof, per_kernel = kernel_roofline(run, dt, args.steps, grmhd, torch)
        # the 2-D blast wave (512^2, PPM + SSP3) as a second plain-path point
        sb = W.blast_wave(512, eta=1e-6)
        rb = grmhd.Run(sb, device="cuda:0")
        dtb = rb.dt()
        for _ in range(args.warmup):
            rb.step(dtb)
        msb = time_steps(rb, dtb, args.steps, torch)
        extra.update({"blast_512sq_ssp3_zone_cycles_per_s": round(sb.ncells * args.steps / (msb * 1e-3), 1),
                      "blast_512sq_ms_per_step": round(msb / args.steps, 4), "per_kernel": per_kernel})
    if args.copy_ref:
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        extra["copy_ref_bytes"] = 2 * a.numel() * 8
    out = {
        "metric": "zone-cycles/s per IMEX-RK step FP64 (plain single grid)",
        "value": round(value, 1),
        "unit": "zone-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "tov_star_cowling_%d^3_ppm_hll_uct_imex_ssp3_433" % args.n,
                   "cells": s.ncells, "grid": [args.n] * 3, "domain": [-12, 12], "eta": "sigma(D) in [1e-6, 1]",
                   "parallelism": "single GPU"},
        "roofline": roof,
        "extra": extra,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(star)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
