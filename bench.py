"""Benchmark of one IMEX-RK step of resistive GRMHD on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (value): the 3-D magnetised polytropic star in a static conformally
flat metric (Cowling), 128^3 cells on [-12, 12]^3, PPM + HLL + upwind CT +
IMEX-SSP3(4,3,3), FP64, seeded synthetic initial data (TOV equilibrium built
by the generator, poloidal field from a vector potential).  A step is one
full pass of the hot path (all IMEX stages and the final recovery).
value = interior cells x timed steps / seconds (zone-cycles/s), inputs
resident in HBM; the step is captured once into a HIP graph and replayed, and
the value is the median of five timed windows of K replays.  Prints one JSON
line.
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
    """eager steps, HIP events on the run's stream; milliseconds"""
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


def capture_step(run, dt, grmhd, torch):
    """one whole step (gr_step) captured into a HIP graph"""
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        grmhd.gr_step(run.grid, run.state, dt, s.cuda_stream)
    torch.cuda.synchronize()
    return g


def time_replays(graph, steps, torch, windows=5):
    """median over `windows` timed windows of `steps` graph replays (HIP
    events on the replay stream); milliseconds per window"""
    s = torch.cuda.Stream()
    out = []
    with torch.cuda.stream(s):
        for _ in range(windows):
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(steps):
                graph.replay()
            e1.record(s)
            e1.synchronize()
            out.append(e0.elapsed_time(e1))
    torch.cuda.synchronize()
    out.sort()
    return out[len(out) // 2], out


def stream_ceiling(grmhd, torch, nbytes=2 << 30, reps=5):
    """the part's practical HBM rate: the library's hand-written streaming
    read and copy (16-byte loads and stores) over nbytes, best of reps"""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    sink = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    s = torch.cuda.current_stream()
    res = {}
    for name, fn, moved in (("read", lambda: grmhd.gr_stream_read(a.data_ptr(), nbytes, sink.data_ptr(), s.cuda_stream),
                             nbytes),
                            ("copy", lambda: grmhd.gr_stream_copy(a.data_ptr(), b.data_ptr(), nbytes, s.cuda_stream),
                             2 * nbytes)):
        fn()
        best = None
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            fn()
            e1.record(s)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        res[name + "_GBps"] = round(moved / (best * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.synchronize()
    res["bytes"] = nbytes
    return res


def csrc_digest():
    """first 16 hex digits of the SHA-256 of the kernel sources"""
    import glob
    import hashlib
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2110_03732_amd", "csrc", "*")))
    return hashlib.sha256(b"".join(open(f, "rb").read() for f in files)).hexdigest()[:16]


def profiled_value(pattern, key, kernel):
    """a per-launch figure of `kernel` from a committed counter summary
    (profiles/<pattern>), or None when the kernel sources changed since the
    counters were taken"""
    import glob
    import re
    for f in glob.glob(os.path.join(ROOT, "profiles", pattern)):
        txt = open(f).read()
        m = re.search(r"csrc-sha256-16: ([0-9a-f]+)", txt)
        t = re.search(r"%s %s: ([0-9.]+)" % (re.escape(key), re.escape(kernel)), txt)
        if m and t and m.group(1) == csrc_digest():
            return float(t.group(1))
    return None


def profiled_traffic(kernel):
    """HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)"""
    return profiled_value("*hbm_traffic.md", "traffic-bytes-per-launch", kernel)


def profiled_step_traffic(per_kernel):
    """counted HBM bytes per step: the per-launch traffic of every kernel
    class times its launches per step, or None if any class is missing or
    the sources changed since the counters were taken"""
    tot = 0.0
    for k, v in per_kernel.items():
        tr = profiled_value("*hbm_traffic.md", "traffic-bytes-per-step", k)
        if tr is None:
            return None
        tot += tr
    return tot


def profiled_fp64_flop(kernel):
    """FP64 flops per launch (rocprofv3 SQ_INSTS_VALU_*_F64)"""
    return profiled_value("*fp64_valu*.md", "fp64-flop-per-launch", kernel)


def fp64_rate(kernel, avg_us):
    """the FP64 VALU side of the roofline: counted flops per launch (from
    the committed counter summary) over the live average launch time"""
    fl = profiled_fp64_flop(kernel)
    if fl is None:
        return None
    tf = fl / (avg_us * 1e-6) / 1e12
    return {"achieved": round(tf, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(tf / FP64_PEAK_TFLOPS, 4),
            "flop_per_launch": fl}


def kernel_roofline(run, dt, steps, grmhd, torch):
    """the timed steps again with every launch of each kernel class
    bracketed by HIP events on the stream it is launched on (while the events
    record, the library runs each pass on one stream, so every class is
    timed alone); roofline of the class with the largest time"""
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
    step_bytes = sum(v[2] for v in per.values()) / steps
    ms, n, by = per[name]
    achieved = by / (ms * 1e-3) / 1e9
    return name, {
        "bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": profiled_traffic(name), "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
        "avg_launch_us": round(ms * 1e3 / n, 2), "launches": n, "alg_bytes_per_launch": by / n,
        "fp64": fp64_rate(name, ms * 1e3 / n),
    }, {k: {"ms_per_step": round(v[0] / steps, 4), "launches_per_step": v[1] / steps,
            "alg_GBps": round(v[2] / (v[0] * 1e-3) / 1e9, 1)} for k, v in per.items()}, step_bytes


def cleaning(run, grmhd, torch, ms_per_step, vcycles=(1, 2, 8)):
    """elliptic divergence cleaning of the run's face fields (gr_clean_divB):
    the divergence norms before and after, and the time of the cleaning alone
    (no norms), eager and as a replayed captured graph, median of 5"""
    out = {}
    s = torch.cuda.current_stream()
    for vc in vcycles:
        before, after = run.clean_divB(vc)
        times = {}
        for mode in ("eager", "graph"):
            if mode == "graph":
                g = torch.cuda.CUDAGraph()
                cs = torch.cuda.Stream()
                torch.cuda.synchronize()
                with torch.cuda.graph(g, stream=cs):
                    grmhd.gr_clean_divB(run.grid, run.state, vc, 0, cs.cuda_stream)
                fn = g.replay
            else:
                def fn():
                    grmhd.gr_clean_divB(run.grid, run.state, vc, 0, s.cuda_stream)
            fn()
            ts = []
            for _ in range(5):
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                e1.synchronize()
                ts.append(e0.elapsed_time(e1))
            ts.sort()
            times[mode] = round(ts[2], 4)
        out["%d_vcycles" % vc] = {"ms_eager": times["eager"], "ms_graph": times["graph"],
                                 "of_a_step_graph": round(times["graph"] / ms_per_step, 3),
                                 "divB_L1_before": float(before[0]), "divB_L1_after": float(after[0]),
                                 "divB_linf_before": float(before[2]), "divB_linf_after": float(after[2])}
    return out


def batched_vs_plain(torch, W, grmhd, nruns, steps, seed=1):
    """The mix of independent runs (1-D shock tubes N in 128..4096 with
    minmod, 2-D blast waves 64^2..256^2 with PPM, eta log-uniform in
    [1e-6, 1], IMEX-SSP2, each run its own dt), `steps` steps each: plain
    per-run launches one run after another on one stream and spread over 8
    streams, against the batch (tiles from the autotuner) launched eagerly and
    as one captured graph per step."""
    prm = W.batch_mix_params(nruns, seed=seed)
    setups = [W.make_run_setup(p, imex=W.SSP2) for p in prm]
    zc = float(sum(s.ncells for s in setups)) * steps
    out = {"runs": nruns, "steps": steps, "cells": int(sum(s.ncells for s in setups)),
           "kinds": {"shock_tube_1d": sum(p["kind"] == "shock_tube" for p in prm),
                     "blast_wave_2d": sum(p["kind"] == "blast_wave" for p in prm)}}

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    runs = [grmhd.Run(s, device="cuda:0") for s in setups]
    dts = [r.dt() for r in runs]

    def plain_one_stream():
        for r, dt in zip(runs, dts):
            for _ in range(steps):
                r.step(dt)
    plain_one_stream_t = timed(plain_one_stream)
    streams = [torch.cuda.Stream() for _ in range(8)]
    runs8 = [grmhd.Run(s, device="cuda:0", stream=streams[i % 8]) for i, s in enumerate(setups)]

    def plain_eight_streams():
        for r, dt in zip(runs8, dts):
            for _ in range(steps):
                r.step(dt)
    plain_eight_t = timed(plain_eight_streams)
    del runs8
    t0 = time.perf_counter()
    b = grmhd.Batch(runs, dts, tune_cache="")
    tune_s = time.perf_counter() - t0
    launches, alg_bytes, _ = b.stats()
    eager_t = timed(lambda: [b.step() for _ in range(steps)])
    b.run(1)  # capture
    graph_t = timed(lambda: b.run(steps))
    tiles = {}
    for i, p in enumerate(prm):
        key = "1d" if p["kind"] == "shock_tube" else "2d"
        tiles[key] = b.tiles(i)[0]
    b.close()
    out.update({
        "plain_1stream_zone_cycles_per_s": round(zc / plain_one_stream_t, 1),
        "plain_8streams_zone_cycles_per_s": round(zc / plain_eight_t, 1),
        "batched_eager_zone_cycles_per_s": round(zc / eager_t, 1),
        "batched_graph_zone_cycles_per_s": round(zc / graph_t, 1),
        "batched_over_plain_1stream": round(plain_one_stream_t / graph_t, 2),
        "batched_over_plain_8streams": round(plain_eight_t / graph_t, 2),
        "batched_launches_per_step": launches,
        "batched_alg_GBps": round(alg_bytes * steps / graph_t / 1e9, 1),
        "autotune_s": round(tune_s, 3), "tiles": tiles})
    return out


def served(torch, W, grmhd, nreq, rate, budgets_gib, seed=7, sweep_rates=(25.0, 50.0, 100.0, 200.0),
           sweep_requests=48, low_rates=(2.0, 5.0, 10.0), low_requests=24):
    """Poisson stream of 2-D blast waves (64^2..512^2) and 3-D stars
    (32^3..96^3), PPM + IMEX-SSP3, 10..500 steps, eta log-uniform; the
    requests' initial data is built before the clock starts (it arrives with
    the request).  For each HBM budget: the continuous-batching loop; then the
    same requests one after another through the plain path."""
    from paper_2110_03732_amd import serve
    trace = W.served_trace(nreq, rate=rate, seed=seed)
    cache = {}

    def payload(req):
        if req["rid"] not in cache:
            cache[req["rid"]] = W.make_run_setup(req, imex=W.SSP3)
        return cache[req["rid"]]
    for r in trace:
        payload(r)
    out = {"requests": nreq, "rate_per_s": rate,
           "mix": {"blast_wave_2d": sum(r["kind"] == "blast_wave" for r in trace),
                   "tov_star_3d": sum(r["kind"] == "tov_star" for r in trace)}}
    for gib in budgets_gib:
        srv = serve.Server(int(gib * (1 << 30)), chunk=4)
        recs, summ = srv.serve(trace, payload)
        out["budget_%gGiB" % gib] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in summ.items()}
    # arrival-rate sweep on the first requests of the same trace (32 GiB)
    sweep = {}
    for r in sweep_rates:
        tr = W.served_trace(sweep_requests, rate=r, seed=seed)
        srv = serve.Server(32 << 30, chunk=4)
        _, summ = srv.serve(tr, payload)
        sweep["%g" % r] = {k: round(summ[k], 4) for k in ("offered_zone_cycles_per_s", "served_zone_cycles_per_s",
                                                          "p50_latency_s", "p99_latency_s", "makespan_s")}
    out["rate_sweep_%d_requests" % sweep_requests] = sweep
    # below capacity: offered load under the served rate, latency without a queue
    low = {}
    for r in low_rates:
        tr = W.served_trace(low_requests, rate=r, seed=seed)
        srv = serve.Server(32 << 30, chunk=4)
        _, summ = srv.serve(tr, payload)
        low["%g" % r] = {k: round(summ[k], 4) for k in ("offered_zone_cycles_per_s", "served_zone_cycles_per_s",
                                                        "p50_latency_s", "p99_latency_s", "makespan_s")}
    out["below_capacity_%d_requests" % low_requests] = low
    # plain path, requests back to back
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    zc = 0.0
    for r in trace:
        s = payload(r)
        run = grmhd.Run(s, device="cuda:0")
        dt = run.dt()
        for _ in range(r["steps"]):
            run.step(dt)
        zc += s.ncells * r["steps"]
        del run
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["plain_sequential_zone_cycles_per_s"] = round(zc / el, 1)
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(setup_fn, small_fn):
    """the oracle as it stands on the host cores: whole IMEX-SSP3 steps of
    the benchmark's own star until about 10 s of work (all threads), and one
    step of the same star at 64^3 on one thread; the thread counts are the
    ones the oracle's OpenMP runtime reports"""
    import oracle

    def sample(s, min_s, max_steps):
        st = oracle.OracleState(s)
        dt = st.dt()
        t0 = time.time()
        steps = 0
        while steps < max_steps and (steps == 0 or time.time() - t0 < min_s):
            st.step(dt)
            steps += 1
        return steps, time.time() - t0

    cores = oracle.threads(0)
    s = setup_fn()
    steps, el = sample(s, 10.0, 5)
    s1 = small_fn()
    oracle.threads(1)
    steps1, el1 = sample(s1, 0.0, 1)
    oracle.threads(cores)
    return {"value": round(s.ncells * steps / el, 1), "unit": "zone-cycles/s", "cores": cores, "kind": "oracle",
            "sample": "%d full IMEX-SSP3 step(s) of the same %dx%dx%d star (%.1f s, OpenMP threads=%d)" % (
                steps, s.n[0], s.n[1], s.n[2], el, cores),
            "one_core": {"value": round(s1.ncells * steps1 / el1, 1), "cores": 1,
                         "sample": "%d step of the star at %dx%dx%d on one thread (%.1f s)" % (
                             steps1, s1.n[0], s1.n[1], s1.n[2], el1)},
            "cpu_model": cpu_model(), "host_threads": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=128, help="cells per direction of the star workload")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extra", action="store_true", help="star workload only (no 2-D point, no roofline replay)")
    ap.add_argument("--no-many", action="store_true", help="skip the batched and served comparisons")
    ap.add_argument("--no-serve", action="store_true", help="skip the served comparison")
    ap.add_argument("--batch-runs", type=int, default=256, help="runs in the batched-vs-plain comparison")
    ap.add_argument("--batch-steps", type=int, default=50)
    ap.add_argument("--serve-requests", type=int, default=160)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--copy-ref", action="store_true",
                    help="end with a 256 MiB streaming copy and read, the reference kernels for scaling HBM counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one MI355X only; runs on more than one GPU are not supported "
              "(independent runs would shard by whole runs; no multi-GPU path is built)", file=sys.stderr)
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
    ms_eager = time_steps(run, dt, args.steps, torch)
    graph = capture_step(run, dt, grmhd, torch)
    graph.replay()
    ms, windows = time_replays(graph, args.steps, torch)
    ms_per_step = ms / args.steps
    value = s.ncells * args.steps / (ms * 1e-3)
    fails = run.fail_count()
    div = run.divB()
    extra = {"recovery_failures": int(fails), "divB_linf": float(div[2]),
             "timing": "median of 5 windows of %d replays of a captured step graph" % args.steps,
             "window_ms": [round(w, 3) for w in windows],
             "eager_ms_per_step": round(ms_eager / args.steps, 4)}
    # elliptic cleaning of the star's face fields after the timed steps
    extra["clean_divB"] = cleaning(run, grmhd, torch, ms_per_step)
    roof = None
    if not args.no_extra:
        kname, roof, per_kernel, step_bytes = kernel_roofline(run, dt, args.steps, grmhd, torch)
        ceil = stream_ceiling(grmhd, torch)
        # the step's algorithmic bytes: every live field read once and every
        # output written once per IMEX pass (243 doubles per cell for
        # IMEX-SSP3 with the metric; 218 with the two point-wise passes as one
        # launch and the stored terms folded as the library stores them)
        alg = 243 * 8.0 * s.ncells
        alg218 = 218 * 8.0 * s.ncells
        gbs = alg / (ms_per_step * 1e-3) / 1e9
        counted = profiled_step_traffic(per_kernel)
        roof["step"] = {
            "alg_bytes_per_step": alg,
            "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "alg_bytes_per_step_218": alg218,
            "frac_218": round(alg218 / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "launch_bytes_per_step": step_bytes,
            "launch_bytes_note": "each launch's own inputs read once and outputs written once, summed over the "
                                 "step's launches: includes the intermediates between kernels",
            "counted_bytes_per_step": counted,
            "counted_over_alg": round(counted / alg, 3) if counted else None,
            "stream_ceiling": ceil,
            "frac_of_copy_ceiling": round(gbs / ceil["copy_GBps"], 4)}
        # the 2-D blast wave (512^2, PPM + SSP3) as a second plain-path point
        sb = W.blast_wave(512, eta=1e-6)
        rb = grmhd.Run(sb, device="cuda:0")
        dtb = rb.dt()
        for _ in range(args.warmup):
            rb.step(dtb)
        msb = time_steps(rb, dtb, args.steps, torch)
        extra.update({"blast_512sq_ssp3_zone_cycles_per_s": round(sb.ncells * args.steps / (msb * 1e-3), 1),
                      "blast_512sq_ms_per_step": round(msb / args.steps, 4), "per_kernel": per_kernel})
        del rb
    if not args.no_extra and not args.no_many:
        print("bench: batched vs plain", file=sys.stderr, flush=True)
        extra["batched"] = batched_vs_plain(torch, W, grmhd, args.batch_runs, args.batch_steps)
        if not args.no_serve:
            print("bench: served", file=sys.stderr, flush=True)
            extra["served"] = served(torch, W, grmhd, args.serve_requests, args.serve_rate, (32.0, 2.0))
    if args.copy_ref:
        # reference kernels of known traffic for scaling the HBM counters:
        # the library's streaming copy and read of 256 MiB
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        sink = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        torch.cuda.synchronize()
        cs = torch.cuda.current_stream().cuda_stream
        grmhd.gr_stream_copy(a.data_ptr(), b.data_ptr(), a.numel() * 8, cs)
        grmhd.gr_stream_read(a.data_ptr(), a.numel() * 8, sink.data_ptr(), cs)
        torch.cuda.synchronize()
        extra["copy_ref_bytes"] = {"k_stream_copy": 2 * a.numel() * 8, "k_stream_read": a.numel() * 8}
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
        out["cpu_baseline"] = cpu_baseline(star, lambda: W.tov_star(64))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
