"""Benchmark: rigid-aggregate Stokesian dynamics time steps on one MI355X.

A step is one pass of the whole hot path over a suspension: neighbour lists,
lubrication and preconditioner set-up, the right-hand side, the GMRES saddle
solve (PSE mobility, lubrication, rigid constraints, block-triangular
preconditioner) and the explicit Euler update.

The default workload is the batched form: 64 independent periodic suspensions of
200-4000 beads (random-sticking clusters of 4-30 beads, phi 0.02-0.25, simple shear
with lubrication, xi = 25/L, tolerance 1e-5), stepped together in mixed precision
(FP32 operator, FP64 Krylov and residual) with multi-system launches.  The same run
times the plain path on the same systems, FP64 and one system at a time, and reports
the ratio.  Every counted solve meets 1e-5 on its FP64 true residual.  GMRES starts
each solve from the linear extrapolation of the two previous steps' solutions in both
(--warm-mode, --cold for zero).  The 256x8 and 4096x20 cluster workloads ride along
as sub-objects (--no-sub to skip).

Prints one JSON line.  --gpus above 1 is not supported: this build runs on a single GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "bead-solves/s at 1e-5 saddle residual vs plain FP64; p50/p99 solve latency"
PEAK_HBM_GBS = 8000.0


# kernel behind each timer class (rocprofv3 names), for matching the two measurements
KERNEL_OF = {"real_sum": "k_real_sum", "spread": "k_spread_fused", "fft_first": "k_fft_lines<2>",
             "fft_y": "k_fft_lines<1>", "fft_green": "k_fft_xgreen", "fft_last": "k_fft_lines<2>",
             "interp": "k_interp", "rigid_lub": "k_agg_lub", "precond": "k_precond_fused",
             "cgs_dot": "k_cgs_chain<0>", "cgs_update": "k_cgs_chain<1>", "cgs_norm_arnoldi": "k_cgs_chain<2>"}


def batch_kernel_names(prec):
    """rocprofv3 names of the multi-system kernels behind each timer class."""
    R = "float" if prec else "double"
    return {"real_sum": f"kb_real<{R}>", "spread": f"kb_spread<{R}>", "fft_first": f"kb_fft<{R}, 0>",
            "fft_y": f"kb_fft<{R}, 1>", "fft_green": f"kb_fft<{R}, 2>", "fft_last": f"kb_fft<{R}, 4>",
            "interp": f"kb_interp<{R}>", "rigid_lub": "kb_agg", "precond": "kb_precond",
            "cgs_dot": "kb_cgs<0>", "cgs_update": "kb_cgs<1>", "cgs_norm_arnoldi": "kb_cgs<2>"}


def progress(msg):
    """Progress line on stderr (the JSON result is the only line on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_table(timers, steps, names=None):
    """Per timer class: ms per step, launches, average launch duration and the
    algorithmic HBM bandwidth (algorithmic bytes of the launches / their time)."""
    names = names or KERNEL_OF
    out = {}
    for k, (ms, n, by) in timers.items():
        if n == 0:
            continue
        out[k] = {"kernel": names.get(k, k), "ms_per_step": round(ms / steps, 4), "launches": n,
                  "avg_us": round(1e3 * ms / n, 2), "alg_bytes_per_launch": int(by / n),
                  "alg_GBps": round(by / (ms * 1e-3) / 1e9, 1) if ms > 0 else None}
    return out


# source file of each kernel, whose hash the counter summaries record
SOURCE_OF = {"kb_fft<float, 2>": "k_mobility.hip", "kb_fft<float, 0>": "k_mobility.hip",
             "kb_fft<float, 1>": "k_mobility.hip", "kb_fft<float, 4>": "k_mobility.hip",
             "kb_spread<float>": "k_mobility.hip", "kb_interp<float>": "k_mobility.hip",
             "k_real_sum": "k_mobility.hip", "k_spread_fused": "k_mobility.hip", "k_spread_split": "k_mobility.hip", "k_fft_lines<1>": "k_mobility.hip",
             "k_fft_lines<2>": "k_mobility.hip", "k_fft_xgreen": "k_mobility.hip", "k_interp": "k_mobility.hip",
             "k_agg_lub": "k_solver.hip", "k_precond_fused": "k_solver.hip", "k_cgs_chain<0>": "k_solver.hip",
             "k_cgs_chain<1>": "k_solver.hip", "k_cgs_chain<2>": "k_solver.hip"}


def measured_traffic(counters_file, kernel):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for a copy of known size),
    or None when there is no summary or the kernel's source file differs from the one
    the counters were taken with."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", counters_file)
    src = SOURCE_OF.get(kernel)
    if not src or not os.path.exists(path):
        return None
    text = open(path).read()
    # every source the summary lists (the kernel's file and the headers it includes) must
    # be the one the counters were taken with
    recorded = dict(re.findall(r"^source (\S+) sha256 ([0-9a-f]{64})$", text, re.M))
    row = re.search(r"^traffic %s (\d+)$" % re.escape(kernel), text, re.M)
    if src not in recorded or not row:
        return None
    for name, digest in recorded.items():
        fn = os.path.join(ROOT, "paper_2607_25161_amd", "csrc", name)
        if not os.path.exists(fn):
            return None
        with open(fn, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return int(row.group(1))


REPLAYABLE = ("real_sum", "spread", "fft_first", "fft_y", "fft_green", "fft_last", "interp", "rigid_lub", "precond")


def dominant(table):
    """Timer class with the largest total time."""
    return max(table, key=lambda k: table[k]["ms_per_step"])


def replay_ms(sysm, table, reps=200):
    """Average launch duration of the dominant kernel, replayed back to back between one
    pair of HIP events on the library stream (None when that class has no replay)."""
    name = dominant(table)
    return sysm.time_kernel(name, reps) if name in REPLAYABLE else None


def roofline_of(table, counters_file=None, launch_ms=None, launch_bytes=None):
    """Dominant kernel against the HBM roofline: algorithmic bytes per launch over the
    average launch duration (from the back-to-back replay when given, else from the
    eager pass's per-launch events, which include each launch's dispatch).  A replay of
    a multi-system launch over every system gives its own bytes per launch."""
    name = dominant(table)
    r = dict(table[name])
    if launch_bytes:
        r["alg_bytes_per_launch"] = int(launch_bytes)
    us = 1e3 * launch_ms if launch_ms else r["avg_us"]
    ach = round(r["alg_bytes_per_launch"] / (us * 1e-6) / 1e9, 1)
    traffic = measured_traffic(counters_file, r["kernel"]) if counters_file else None
    return {"bound": "hbm", "kernel": r["kernel"], "timer": name, "achieved": ach, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": traffic,
            "alg_bytes_per_launch": r["alg_bytes_per_launch"], "avg_launch_us": round(us, 2),
            "duration_from": "back-to-back replay, HIP events" if launch_ms else "eager pass, HIP events per launch",
            "eager_event_avg_us": r["avg_us"]}


def _oracle_cores():
    try:
        from threadpoolctl import threadpool_info
        return int(max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count()]))
    except Exception:
        return int(os.cpu_count())


def cpu_baseline(precision_note):
    """Time the CPU oracle on a bounded sample of the same generator (one solve)."""
    import fsdgen
    from oracle import saddle
    s = fsdgen.sheared_clusters(n_agg=96, n_b=8, phi=0.10, name="clusters-96x8")
    t0 = time.perf_counter()
    U, F, res, A = saddle.solve_suspension(s)
    dt = time.perf_counter() - t0
    return {"value": s.n_bead / dt, "unit": "bead-solves/s", "cores": _oracle_cores(), "kind": "oracle",
            "sample": f"1 dense FP64 solve of 96x8 clusters ({s.n_bead} beads, phi 0.10, shear + lubrication, "
                      f"same generator) in {dt:.1f} s; {precision_note}"}


def cpu_baseline_uneven(systems, picks=(17, 3)):
    """The oracle on a bounded sample of the batched workload: one dense FP64 solve of each
    picked system, as a rate over their beads."""
    from oracle import saddle
    t0 = time.perf_counter()
    nb = 0
    for k in picks:
        saddle.solve_suspension(systems[k])
        nb += systems[k].n_bead
    dt = time.perf_counter() - t0
    return {"value": nb / dt, "unit": "bead-solves/s", "cores": _oracle_cores(), "kind": "oracle",
            "sample": f"1 dense FP64 solve each of uneven systems {list(picks)} "
                      f"({', '.join(str(systems[k].n_bead) for k in picks)} beads) in {dt:.1f} s"}


def _sync():
    import torch
    torch.cuda.synchronize()


def run_plain(F, systems, steps, warm, graphs=True):
    """Plain path: FP64, one system at a time (each system's step after the last one's)."""
    sys_ = [F.System.from_suspension(s0) for s0 in systems]
    for s in sys_:
        s.set_warm_start(warm)
        if not graphs:
            s.set_graphs(False)
    for s in sys_:          # warm-up: lists sized, graphs captured
        s.step(1e-3, 1)
    _sync()
    t0 = time.perf_counter()
    ok, its = 0, []
    for _ in range(steps):
        for s in sys_:
            info = s.step(1e-3, 1)
            its.append(info.iterations)
            ok += s.n_bead if (info.status == 0 and info.rel_residual_fp64 <= 1e-5) else 0
    _sync()
    dt_ = time.perf_counter() - t0
    for s in sys_:
        s.close()
    return {"value": round(ok / dt_, 1), "ms_per_step": round(1e3 * dt_ / steps, 3),
            "gmres_iterations_mean": round(float(np.mean(its)), 2), "graphs": graphs, "steps": steps}


def tuned_xi(F, systems, precision):
    """Per system, the measured fastest splitting parameter between the two fixed policies
    of Section 3.2 (0.5/a and 25/L), in the given precision."""
    out = []
    for s0 in systems:
        probe = F.System.from_suspension(s0, precision=precision)
        lo, hi = sorted((0.5 / s0.a, 25.0 / s0.L))
        xi, _ = probe.autotune_xi(lo, hi, 5)
        probe.close()
        out.append(xi)
    return out


def run_plain_xi(F, systems, steps, warm, xis):
    """The plain path (eager launches) at given splitting parameters."""
    import dataclasses
    return run_plain(F, [dataclasses.replace(s0, xi=xi) for s0, xi in zip(systems, xis)], steps, warm, graphs=False)


def run_batch(F, systems, steps, warmup, warm, precision, fused=True, timing=False, replay=None, xis=None,
              tiles=False):
    """All systems admitted to one batch and stepped together; returns the figures, the
    per-step latencies and, with timing, the kernel table and the replayed dominant launch.
    xis: a splitting parameter per system (default: the workload's own); tiles: measure
    each system's transform tiles first."""
    sys_ = [F.System.from_suspension(s0, precision=precision, **({"xi": xis[k]} if xis else {}))
            for k, s0 in enumerate(systems)]
    chosen = [s.autotune_tiles(10) for s in sys_] if tiles else None
    for s in sys_:
        s.set_warm_start(warm)
    b = F.Batch(1 << 40, len(sys_))
    b.set_fused(fused)
    slots = [b.admit(s) for s in sys_]
    # a multi-system launch reserves its largest system's LDS for every workgroup: measure
    # the caps on the systems' transform tiles that make the shared launches fastest
    caps = b.autotune_tiles(10) if fused else None
    for _ in range(warmup):
        b.step(1e-3)
    _sync()
    lat, its = [], []
    ok = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        b.step(1e-3)
        lat.append(time.perf_counter() - a)
        for k, sl in enumerate(slots):
            inf = b.info(sl)
            its.append(inf.iterations)
            ok += sys_[k].n_bead if (inf.status == 0 and inf.rel_residual_fp64 <= 1e-5) else 0
    _sync()
    dt_ = time.perf_counter() - t0
    out = {"value": round(ok / dt_, 1), "ms_per_step": round(1e3 * dt_ / steps, 3),
           "gmres_iterations_mean": round(float(np.mean(its)), 2), "gmres_iterations_max": int(np.max(its)),
           "lat": lat}
    if chosen:
        out["tiles"] = {f"B{b} G{g}": sum(1 for c in chosen if c == (b, g)) for b, g in sorted(set(chosen))}
    if caps:
        out["lds_caps_kb"] = {"lines": caps[0] // 1024 or None, "x_green": caps[1] // 1024 or None}
    if timing:
        # the same kernels once more, one more step with event timing on every launch
        b.set_timing(True)
        b.step(1e-3)
        out["table"] = kernel_table(b.timers(), 1, batch_kernel_names(precision == F.FSD_MIXED))
        b.set_timing(False)
        name = dominant(out["table"])
        if replay:
            # the largest kernels replayed back to back, each over every system: whichever
            # of them ends up dominant, its launch time and a profile of the same run agree
            top = sorted(out["table"], key=lambda k: -out["table"][k]["ms_per_step"])[:4]
            for k in top:
                if k in REPLAYABLE:
                    ms, by = b.time_kernel(k, replay)
                    out["table"][k]["replay_us"] = round(1e3 * ms, 2)
                    out["table"][k]["replay_alg_bytes"] = int(by)
                    if k == name:
                        out["replay"] = (ms, by)
    b.close()
    for s in sys_:
        s.close()
    return out


def bench_batched(args, F, fsdgen, torch):
    """Uneven systems: the mixed-precision batch against the plain FP64 path."""
    systems = fsdgen.uneven_systems(n_sys=args.systems)
    n_tot = sum(s.n_bead for s in systems)
    warm = 0 if args.cold else args.warm_mode
    progress(f"generated {len(systems)} systems, {n_tot} beads")
    plain_steps = max(1, args.steps // 2)
    only = args.headline_only  # profiling runs: the measured batch alone
    plain = plain_g = None
    if not only:
        plain = run_plain(F, systems, plain_steps, warm, graphs=False)
        progress(f"plain FP64 one at a time (eager launches): {plain['value']} bead-solves/s")
        plain_g = run_plain(F, systems, plain_steps, warm, graphs=True)
        progress(f"plain FP64 one at a time (captured graphs): {plain_g['value']} bead-solves/s")
    # the batched form: splitting parameter and transform tiles measured per system
    t0 = time.perf_counter()
    xis = tuned_xi(F, systems, F.FSD_MIXED)
    t_tune = time.perf_counter() - t0
    mixed = run_batch(F, systems, args.steps, args.warmup, warm, F.FSD_MIXED, fused=True, timing=True, replay=50,
                      xis=xis, tiles=True)
    progress(f"batched mixed, measured xi and tiles: {mixed['value']} bead-solves/s (xi tuning {t_tune:.1f} s)")
    paper = b64 = streams = plain_t = None
    if not only:
        paper = run_batch(F, systems, plain_steps, 1, warm, F.FSD_MIXED, fused=True)
        progress(f"batched mixed at xi = 25/L: {paper['value']} bead-solves/s")
        b64 = run_batch(F, systems, plain_steps, 1, warm, F.FSD_FP64, fused=True)
        progress(f"batched FP64 at xi = 25/L: {b64['value']} bead-solves/s")
        streams = run_batch(F, systems, plain_steps, 1, warm, F.FSD_MIXED, fused=False, xis=xis)
        progress(f"batched mixed, one stream per system, measured xi: {streams['value']} bead-solves/s")
        plain_t = run_plain_xi(F, systems, plain_steps, warm, xis)
        progress(f"plain FP64 one at a time at the measured xi: {plain_t['value']} bead-solves/s")
    grids = sorted({int(F.System.from_suspension(systems[k], xi=xis[k]).info().grid) for k in range(len(systems))})
    table = mixed["table"]
    rep = mixed.get("replay")
    roofline = roofline_of(table, "hbm_counters_uneven-64_mixed.md", rep[0] if rep else None,
                           rep[1] if rep else None)
    roofline["launch"] = f"one multi-system launch over all {len(systems)} systems"
    lat = mixed["lat"]
    ctx = lambda r: None if r is None else {k: v for k, v in r.items() if k not in ("lat", "table", "replay")}
    out = {
        "metric": METRIC, "value": mixed["value"], "unit": "bead-solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 operator / f64 Krylov", "data": "synthetic",
        "config": {"workload": f"{len(systems)} independent sheared cluster suspensions, 200-4000 beads "
                               f"(4-30 per aggregate), phi 0.02-0.25, tol 1e-5; batched, mixed precision, "
                               f"splitting parameter and transform tiles measured per system",
                   "n_bead_total": n_tot, "grids": grids, "xi_range": [round(min(xis), 4), round(max(xis), 4)],
                   "precision": "mixed", "warm_start": warm, "parallelism": "single GPU, multi-system launches"},
        "latency_ms": {"p50": round(1e3 * float(np.percentile(lat, 50)), 3),
                       "p99": round(1e3 * float(np.percentile(lat, 99)), 3),
                       "what": "per solve: every system's solve completes within its batched step"},
        "speedup_vs_plain": round(mixed["value"] / plain["value"], 3) if plain else None,
        "speedup_vs_plain_graphed": round(mixed["value"] / plain_g["value"], 3) if plain_g else None,
        "plain": "FP64, one system at a time, xi = 25/L (the workload's policy), eager launches",
        "gmres_iterations_mean": mixed["gmres_iterations_mean"], "gmres_iterations_max": mixed["gmres_iterations_max"],
        "tiles": mixed.get("tiles"), "lds_caps_kb": mixed.get("lds_caps_kb"), "xi_tuning_s": round(t_tune, 2),
        "plain_fp64_one_at_a_time": plain, "plain_fp64_one_at_a_time_graphed": plain_g,
        "plain_fp64_one_at_a_time_measured_xi": plain_t,
        "batched_mixed_xi_25_over_L": ctx(paper), "batched_fp64_xi_25_over_L": ctx(b64),
        "batched_mixed_streams_measured_xi": ctx(streams),
        "kernels": table,
        "kernel_timing": ("HIP events around every multi-system launch of one extra step on the batch stream, "
                          "bytes of the systems still iterating in each launch"),
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_uneven(systems)
        progress("cpu baseline done")
    if not args.no_sub:
        out["sub"] = {"clusters-256x8": bench_clusters(args, F, fsdgen, torch, emit=False)}
        progress("256x8 sub-run done")
        out["sub"]["clusters-4096x20"] = bench_large(args, F, fsdgen, torch, emit=False, steps=3)
        progress("4096x20 sub-run done")
    print(json.dumps(out), flush=True)


def bench_serving(args, F, fsdgen, torch):
    """Request stream served by the continuous-batching engine: capacity from a closed loop,
    then Poisson arrivals swept over multiples of it; the plain path (FP64, one request at a
    time) serves the same requests for comparison."""
    from paper_2607_25161_amd.serving import BatchEngine, LibBackend, Request, poisson_arrivals
    reqs = fsdgen.serving_requests(args.requests, n_range=(100, args.max_beads), n_steps=args.req_steps, kT=args.kT,
                                   shear_rate=args.shear_rate)
    sheared = args.shear_rate > 0.01  # faster shear needs the sheared lattice's images across the y faces
    args.precision = args.precision or "mixed"
    prec = F.FSD_MIXED if args.precision == "mixed" else F.FSD_FP64
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)

    def run(rate, seed, subset=None, n_steps=args.req_steps, precision=prec, slots=args.slots, multi=8):
        sel = reqs if subset is None else subset
        # Brownian requests: the previous solution, not an extrapolation of noisy ones
        be = LibBackend(F, budget, slots, dict(precision=precision), warm_start=0 if args.cold else 1,
                        lees_edwards=sheared, drift=args.serve_drift)
        eng = BatchEngine(be, max_slots=slots, dt=1e-3, max_steps_per_tick=multi)
        t_arr = np.zeros(len(sel)) if rate is None else poisson_arrivals(np.random.default_rng(seed), len(sel), rate)
        rs = [Request(k, s, n_steps, arrival=float(t_arr[k])) for k, s in enumerate(sel)]

        def tick(e):
            if e.ticks % 5 == 0:
                progress(f"tick {e.ticks}: {len(e.active)} active, {len(e.queue)} queued, {len(e.done)} done")

        rep = eng.run(rs, on_tick=tick)
        torch.cuda.synchronize()
        be.batch.close()
        return rep

    def summary(rep):
        return {"bead_solves_per_s": round(rep["bead_solves_per_s"], 1),
                "p50_ms": round(1e3 * rep["p50_latency_s"], 1) if rep["p50_latency_s"] is not None else None,
                "p99_ms": round(1e3 * rep["p99_latency_s"], 1) if rep["p99_latency_s"] is not None else None,
                "completed": rep["completed"], "failed": rep["failed"], "span_s": round(rep["span_s"], 2)}

    progress(f"generated {len(reqs)} requests, {sum(s.n_bead for s in reqs)} beads")
    if args.warmup:                                 # code objects loaded, first-touch allocations
        run(None, 0, sorted(reqs, key=lambda s: s.n_bead)[:2], 2)
    closed = run(None, 0)                           # every request queued at t = 0: capacity
    progress(f"closed loop: {summary(closed)}")
    cap = closed["completed"] / closed["span_s"]
    rates = {}
    for load in [float(v) for v in args.loads.split(",")]:
        rep = run(load * cap, 1)
        rates[str(load)] = dict(summary(rep), arrival_rate=round(load * cap, 4))
        progress(f"load {load}: {rates[str(load)]}")
    plain = run(None, 0, precision=F.FSD_FP64, slots=1, multi=1)
    progress(f"plain FP64, one request at a time: {summary(plain)}")
    head = rates.get("1.0") or next(iter(rates.values()))
    out = {
        "metric": METRIC, "value": summary(closed)["bead_solves_per_s"], "unit": "bead-solves/s", "n_gpus": 1,
        "steps": args.req_steps, "warmup": args.warmup, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == F.FSD_FP64 else "f32 operator / f64 Krylov", "data": "synthetic",
        "config": {"workload": f"{len(reqs)} requests of {args.req_steps} steps, 100-{args.max_beads} beads "
                               f"(log-uniform), 4-30 beads per aggregate, phi 0.02-0.25, shear rate {args.shear_rate} "
                               f"({'sheared lattice' if sheared else 'cube'}) + lubrication + "
                               f"Brownian kT {args.kT}, drift "
                               f"{['off', 'by random finite differences', 'by Fixman midpoints'][args.serve_drift]}, "
                               f"tol 1e-5, closed loop",
                   "n_bead_total": int(sum(s.n_bead for s in reqs)), "slots": args.slots,
                   "mem_budget_gib": round(budget / 2 ** 30, 1), "precision": args.precision,
                   "warm_start": 0 if args.cold else 1, "parallelism": "single GPU, continuous batching"},
        "latency_ms": {"p50": head["p50_ms"], "p99": head["p99_ms"], "at_load": 1.0 if "1.0" in rates else None},
        "capacity_requests_per_s": round(cap, 4),
        "closed_loop": summary(closed),
        "poisson_loads": rates,
        "plain_fp64_one_at_a_time": summary(plain),
        "speedup_vs_plain": round(closed["bead_solves_per_s"] / plain["bead_solves_per_s"], 3),
        "failed": closed["failed"] + sum(r["failed"] for r in rates.values()),
        "roofline": None,
    }
    print(json.dumps(out), flush=True)


def bench_large(args, F, fsdgen, torch, emit=True, steps=None):
    """81,920 beads (4096 clusters of 20, phi 0.20, 128^3): FP64 against mixed precision."""
    n_steps = steps or args.steps
    s = fsdgen.config(2)
    progress(f"generated {s.name}: {s.n_bead} beads")
    stream = torch.cuda.current_stream().cuda_stream
    res = {}
    for prec_name, prec in (("fp64", F.FSD_FP64), ("mixed", F.FSD_MIXED)):
        sysm = F.System.from_suspension(s, stream=stream, precision=prec)
        sysm.set_warm_start(0 if args.cold else args.warm_mode)
        U0, _, _ = sysm.solve()              # warm-up: lists sized, graphs captured
        torch.cuda.synchronize()
        progress(f"{prec_name}: warm-up solve done")
        lat, its, rr = [], [], []
        t0 = time.perf_counter()
        for _ in range(n_steps):
            a = time.perf_counter()
            si = sysm.step(s.dt, 1)
            lat.append(time.perf_counter() - a)
            its.append(si.iterations)
            rr.append(si.rel_residual_fp64)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        progress(f"{prec_name}: {n_steps} timed steps in {el:.2f} s")
        sysm.set_timing(True)
        sysm.step(s.dt, 1)
        table = kernel_table(sysm.timers(), 1)
        sysm.set_timing(False)
        rep = replay_ms(sysm, table, 20)
        info = sysm.info()
        sysm.close()
        res[prec_name] = {"value": s.n_bead * sum(1 for r in rr if r <= 1e-5) / el, "ms_per_step": 1e3 * el / n_steps,
                          "lat": lat, "its": float(np.mean(its)), "max_res": float(max(rr)), "U0": U0,
                          "table": table, "info": info, "replay": rep}
    m, d = res["mixed"], res["fp64"]
    du = np.linalg.norm(m["U0"][:, :3] - d["U0"][:, :3]) / np.linalg.norm(d["U0"][:, :3])
    dw = np.linalg.norm(m["U0"][:, 3:] - d["U0"][:, 3:]) / np.linalg.norm(d["U0"][:, 3:])
    info = d["info"]
    out = {
        "metric": METRIC, "value": round(m["value"], 1), "unit": "bead-solves/s", "n_gpus": 1,
        "steps": n_steps, "warmup": 1, "ms_per_step": round(m["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 matvec / f64 Krylov", "data": "synthetic",
        "config": {"workload": f"{s.name} clusters in shear + lubrication", "n_bead": s.n_bead, "n_agg": s.n_agg,
                   "phi": round(s.phi, 3), "L": round(s.L, 3), "grid": info.grid, "support": info.support,
                   "xi": info.xi, "r_cut": round(info.r_cut, 3), "nnz_real": int(info.nnz_real), "tol": s.gmres_tol,
                   "precision": "mixed", "warm_start": 0 if args.cold else args.warm_mode, "parallelism": "single GPU"},
        "latency_ms": {"p50": round(1e3 * float(np.percentile(m["lat"], 50)), 3),
                       "p99": round(1e3 * float(np.percentile(m["lat"], 99)), 3)},
        "gmres_iterations_mean": round(m["its"], 2), "max_rel_residual": m["max_res"],
        "fp64": {"value": round(d["value"], 1), "ms_per_step": round(d["ms_per_step"], 3),
                 "gmres_iterations_mean": round(d["its"], 2), "max_rel_residual": d["max_res"],
                 "kernels": d["table"],
                 "roofline": roofline_of(d["table"], f"hbm_counters_{s.name}_fp64.md", launch_ms=d["replay"])},
        "speedup_mixed_vs_fp64": round(m["value"] / d["value"], 3),
        "mixed_vs_fp64_rel_diff": {"U": float(du), "W": float(dw)},
        "kernels": m["table"],
        "roofline": roofline_of(m["table"], f"hbm_counters_{s.name}_mixed.md", launch_ms=m["replay"]),
    }
    if emit:
        print(json.dumps(out), flush=True)
    return out


def bench_rods(args, F, fsdgen, torch):
    """The scaling study of Section 3.2: wall-clock time per step per bead, t_s, of Brownian
    rigid rods (n_b beads each) in a periodic cube, against the total bead count, at the two
    splitting-parameter policies (xi = 0.5/a and xi = 25/L).  Each case times args.rod_steps
    steps after args.rod_warmup discarded ones (the paper: 100 after 10)."""
    args.precision = args.precision or "mixed"
    nbs = [int(v) for v in args.rod_nb.split(",")]
    phis = [float(v) for v in args.rod_phi.split(",")]
    ntots = [int(v) for v in args.rod_ntot.split(",")]
    prec = F.FSD_MIXED if args.precision == "mixed" else F.FSD_FP64
    stream = torch.cuda.current_stream().cuda_stream
    cases = []
    for nb in nbs:
        for phi in phis:
            for nt in ntots:
                for policy in ("fixed", "box"):
                    try:
                        s0 = fsdgen.brownian_rods(max(1, nt // nb), nb, phi, xi_policy=policy)
                    except ValueError as e:  # rods longer than the box
                        progress(f"rods n_b {nb} phi {phi} N_tot {nt}: skipped ({e})")
                        break
                    try:
                        sysm = F.System.from_suspension(s0, stream=stream, precision=prec, gmres_maxit=20000)
                    except F.FsdError as e:  # e.g. a spectral grid above 256 at xi = 0.5/a in a large box
                        progress(f"rods n_b {nb} phi {phi} N_tot {nt} {policy}: skipped ({e})")
                        cases.append({"n_b": nb, "phi": phi, "n_bead": s0.n_bead,
                                      "xi_policy": "0.5/a" if policy == "fixed" else "25/L", "skipped": str(e)})
                        continue
                    sysm.set_pair_forces(k_n=s0.extra["k_n"], r_cut=2.0 * s0.a)
                    sysm.set_warm_start(1)
                    if args.rod_drift:
                        sysm.set_drift(args.rod_drift)
                    info = sysm.info()
                    for _ in range(args.rod_warmup):
                        sysm.step(s0.dt, 1)
                    torch.cuda.synchronize()
                    its, ok = [], 0
                    t0 = time.perf_counter()
                    for _ in range(args.rod_steps):
                        si = sysm.step(s0.dt, 1)
                        its.append(si.iterations)
                        ok += si.status == 0 and si.rel_residual_fp64 <= s0.gmres_tol
                    torch.cuda.synchronize()
                    el = time.perf_counter() - t0
                    sysm.close()
                    c = {"n_b": nb, "phi": phi, "n_bead": s0.n_bead, "n_rod": s0.n_agg, "L": round(s0.L, 2),
                         "xi_policy": "0.5/a" if policy == "fixed" else "25/L", "xi": round(info.xi, 4),
                         "grid": info.grid, "r_cut": round(info.r_cut, 2),
                         "t_s_us": round(1e6 * el / args.rod_steps / s0.n_bead, 4),
                         "ms_per_step": round(1e3 * el / args.rod_steps, 3),
                         "gmres_iterations_mean": round(float(np.mean(its)), 1),
                         "solves_within_tol": f"{ok}/{args.rod_steps}"}
                    cases.append(c)
                    progress(f"rods n_b {nb} phi {phi} N_tot {s0.n_bead} xi {c['xi_policy']}: "
                             f"t_s {c['t_s_us']} us ({c['ms_per_step']} ms per step, grid {info.grid})")
    best = min((c for c in cases if "t_s_us" in c), key=lambda c: c["t_s_us"])
    out = {"metric": "t_s: wall-clock time per time step per bead, Brownian rigid rods (Section 3.2)",
           "value": best["t_s_us"], "unit": "us", "n_gpus": 1, "steps": args.rod_steps,
           "warmup": args.rod_warmup, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if prec == F.FSD_FP64 else "f32 operator / f64 Krylov", "data": "synthetic",
           "config": {"workload": "Brownian rigid rods, Hertz contact, lubrication, tol 1e-5",
                      "drift": ["none", "random finite differences", "Fixman"][args.rod_drift],
                      "precision": args.precision, "parallelism": "single GPU"},
           "cases": cases}
    print(json.dumps(out), flush=True)


def bench_copy(args, torch):
    """Device-to-device copy of 1 GiB: the measured HBM bandwidth next to the 8 TB/s
    vendor figure, and the reference kernel for scaling the FETCH_SIZE / WRITE_SIZE
    counters (2 x 1 GiB of traffic per copy)."""
    n = (1 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(max(1, args.warmup)):
        dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(args.steps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.steps
    gbs = 2 * (1 << 30) / (ms * 1e-3) / 1e9
    print(json.dumps({"metric": "device copy bandwidth", "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
                      "higher_is_better": True, "config": {"workload": "copy of 1 GiB (float64)"},
                      "frac_of_8TBps": round(gbs / PEAK_HBM_GBS, 4)}), flush=True)


def bench_clusters(args, F, fsdgen, torch, emit=True):
    """256 clusters of 8 (2048 beads, phi 0.10, 64^3), FP64 at tol 1e-6 (or --precision)."""
    args.precision = args.precision or "fp64"
    stream = torch.cuda.current_stream()
    s = fsdgen.config(1)
    prec = F.FSD_MIXED if args.precision == "mixed" else F.FSD_FP64
    def timed_run(warm):
        sysm = F.System.from_suspension(s, stream=stream.cuda_stream, precision=prec)
        sysm.set_warm_start(warm)
        for _ in range(args.warmup):
            sysm.step(s.dt, 1)
        info = sysm.info()
        # timed region: graph-replayed GMRES, no instrumentation
        torch.cuda.synchronize()
        lat, its, res = [], [], []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            a = time.perf_counter()
            si = sysm.step(s.dt, 1)
            lat.append(time.perf_counter() - a)
            its.append(si.iterations)
            res.append(si.rel_residual_fp64)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        sysm.close()
        return info, lat, its, res, elapsed

    info, lat, its, res, elapsed = timed_run(0 if args.cold else args.warm_mode)
    cold = None
    if not args.cold:  # the same steps with every solve from zero, for comparison
        _, _, c_its, c_res, c_el = timed_run(0)
        cold = {"value": round(s.n_bead * sum(1 for r in c_res if r <= 1e-5) / c_el, 1),
                "ms_per_step": round(1e3 * c_el / args.steps, 3),
                "gmres_iterations_mean": round(float(np.mean(c_its)), 2)}

    # kernel durations: the same trajectory again from the same start (a fresh system,
    # the same warm-up), with start/stop events carried by every timed launch on the
    # library's stream (this runtime cannot time kernels inside captured graphs, so this
    # pass launches eagerly; the kernels are the same), then the dominant kernel replayed
    # back to back for its launch duration without dispatch gaps
    sysm = F.System.from_suspension(s, stream=stream.cuda_stream, precision=prec)
    sysm.set_warm_start(0 if args.cold else args.warm_mode)
    for _ in range(args.warmup):
        sysm.step(s.dt, 1)
    sysm.set_timing(True)
    for _ in range(args.steps):
        sysm.step(s.dt, 1)
    timers = sysm.timers()
    sysm.set_timing(False)
    table = kernel_table(timers, args.steps)
    rep = replay_ms(sysm, table)
    torch.cuda.synchronize()
    sysm.close()

    counted = sum(1 for r in res if r <= 1e-5)
    value = s.n_bead * counted / elapsed
    roofline = roofline_of(table, f"hbm_counters_{s.name}_{args.precision}.md", rep)
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "bead-solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == F.FSD_FP64 else "f32 matvec / f64 Krylov", "data": "synthetic",
        "config": {"workload": f"{s.name} clusters in shear + lubrication", "n_bead": s.n_bead,
                   "n_agg": s.n_agg, "phi": round(s.phi, 3), "L": round(s.L, 3), "grid": info.grid,
                   "support": info.support, "xi": info.xi, "r_cut": round(info.r_cut, 3), "tol": s.gmres_tol,
                   "precision": args.precision, "warm_start": 0 if args.cold else args.warm_mode, "parallelism": "single GPU"},
        "latency_ms": {"p50": round(1e3 * float(np.percentile(lat, 50)), 3),
                       "p99": round(1e3 * float(np.percentile(lat, 99)), 3)},
        "gmres_iterations_mean": round(float(np.mean(its)), 2),
        "max_rel_residual": float(max(res)),
        "cold_start": cold,
        "kernels": table,
        "kernel_timing": ("start/stop HIP events carried by each timed launch on the library stream, eager pass "
                          "over the same steps from the same start (each interval includes the launch's dispatch)"),
        "roofline": roofline,
    }
    if emit and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline("bead-solves/s of the oracle as it stands")
    if emit:
        print(json.dumps(out), flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default=None,
                    help="clusters: fp64 by default; serving and rods: mixed by default")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["batched", "clusters", "large", "serving", "rods", "copy"],
                    default="batched")
    ap.add_argument("--rod-nb", default="8,27", help="rods: beads per rod")
    ap.add_argument("--rod-phi", default="0.01,0.05,0.10", help="rods: volume fractions")
    ap.add_argument("--rod-ntot", default="2000,8000,32000", help="rods: total bead counts")
    ap.add_argument("--rod-steps", type=int, default=20, help="rods: timed steps per case (the paper: 100)")
    ap.add_argument("--rod-warmup", type=int, default=5, help="rods: discarded steps per case (the paper: 10)")
    ap.add_argument("--rod-drift", type=int, choices=[0, 1, 2], default=2,
                    help="rods: Brownian drift (0 none, 1 random finite differences, 2 Fixman)")
    ap.add_argument("--no-sub", action="store_true", help="batched: skip the 256x8 and 4096x20 sub-runs")
    ap.add_argument("--headline-only", action="store_true",
                    help="batched: the measured mixed batch alone, no plain or other batched forms (for profiling)")
    ap.add_argument("--systems", type=int, default=64)
    ap.add_argument("--requests", type=int, default=8)
    ap.add_argument("--req-steps", type=int, default=20)
    ap.add_argument("--max-beads", type=int, default=50000)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--loads", default="0.25,0.5,1.0,2.0,4.0",
                    help="serving: Poisson arrival rates as multiples of the measured capacity")
    ap.add_argument("--kT", type=float, default=1.0, help="thermal energy of the serving requests")
    ap.add_argument("--serve-drift", type=int, choices=[0, 1, 2], default=0,
                    help="serving: Brownian drift of the requests (0 off, the default: the timed work is the "
                         "solves; 1 random finite differences, 2 Fixman: two more solves per step)")
    ap.add_argument("--shear-rate", type=float, default=1.0,
                    help="shear rate of the serving requests (on the sheared lattice; 0.01 or less keeps the cube)")
    ap.add_argument("--cold", action="store_true",
                    help="GMRES from zero in every solve (default: warm starts; the stopping test is the same)")
    ap.add_argument("--warm-mode", type=int, choices=[1, 2, 3], default=2,
                    help="warm start from the previous solution (1) or the linear (2) or quadratic (3) "
                         "extrapolation of the last solutions")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; this build runs on one GPU "
              f"(independent systems would shard across GPUs by longest-processing-time assignment)", file=sys.stderr)
        sys.exit(2)

    import torch
    import fsdgen
    import paper_2607_25161_amd as F

    torch.cuda.set_device(0)
    if args.workload == "copy":
        return bench_copy(args, torch)
    if args.workload == "batched":
        return bench_batched(args, F, fsdgen, torch)
    if args.workload == "serving":
        return bench_serving(args, F, fsdgen, torch)
    if args.workload == "large":
        return bench_large(args, F, fsdgen, torch)
    if args.workload == "rods":
        return bench_rods(args, F, fsdgen, torch)
    if args.workload == "clusters":
        return bench_clusters(args, F, fsdgen, torch)


if __name__ == "__main__":
    main()
