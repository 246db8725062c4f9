#!/usr/bin/env python3
"""Benchmark of the JFA / dJFA hot path on one MI355X.

Default workload: 8192 x 8192 pixels, 2^20 uniform random seeds, moves in
[-4, 4] per axis (the two maps of a simulation, 2 x 256 MiB, stream from
HBM).  One benchmark step is one simulation time step of the whole path,
run by two twins with the same seed trajectory: the seeds move (on the
device), the JFA twin recomputes its diagram from scratch and the dJFA
twin updates its diagram from the previous step (Alg. 1).  The timed
region runs the JFA twin's K steps, then the dJFA twin's K steps, each as
a lone simulation would run.  Inputs are resident in HBM before the timed
region; nothing leaves the device inside it.

Both label formats (int32 seed IDs and packed 16-bit x/y positions) are
measured, one after the other, and the line reports the faster one, with
the other's figures under "labels".  `value` is pixel-updates/s over the
timed region: width*height*(JFA passes + dJFA passes) per step, divided by
the measured time of both twins' steps (moves, fills and splats included).
Similarity to the exact diagram (Sec. VI-A) is checked outside the timed
region at t = 1, at the end of the timed steps and at the workload's full
length, and for the 512^2 and 4096^2 workloads over their full lengths.
The CPU oracle is timed last, on the host's cores (cpu_baseline).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large]
                  [--label id|xy|both] [--with-djfam] [--no-tune] [--no-cpu]

--with-djfam adds a "djfam" block: a Manhattan-metric dJFA twin (Sec. V-C)
timed in a loop of its own, with T_dJFAe/T_dJFAm and its similarity to the
Euclidean JFA map.
"""
from __future__ import annotations

import argparse
import copy
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pixel-updates/s and ms per time step (dJFA vs JFA), % HBM peak; p50/p99 step latency"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published peak
BYTES_PER_PIXEL_UPDATE = 8     # one 4-byte label read + one 4-byte label write per pass
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2209_00117_amd", "csrc", f)
                  for f in ("vd_device.h", "vd_quad.h", "vd_tail.h", "vd_kernels.hip",
                            "vd_kernels.h", "vd_relabel.hip")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "flood_traffic.json")


def kernel_sha() -> str:
    """Hash of the flood kernels' sources (the traffic record names it)."""
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per flood pass from the committed rocprofv3 counter runs
    (a launch that runs two passes counts as two), or None when they were
    taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    entry = rec.get(workload)
    if not entry or entry.get("kernel_sha") != kernel_sha():
        return None
    return entry.get("bytes_per_pass")


def pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


def host_cpus():
    """CPUs this process may use (what `nproc` prints), the cgroup CPU quota
    if one is set (in cores), and lscpu's model name."""
    nproc = len(os.sched_getaffinity(0))
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, period = f.read().split()[:2]
        if q != "max":
            quota = int(q) / int(period)
    except (OSError, ValueError):
        pass
    model = None
    try:
        text = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in text.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    return nproc, quota, model


def oracle_steps(O, spec, xy, build_threads, threads, steps):
    """The oracle's twins on one workload: VD_0 by its full JFA with
    build_threads (untimed; the dJFA twin starts from a copy), then `steps`
    time steps timed with `threads` threads: move both twins, JFA step of
    one, dJFA step of the other.  Returns per-step seconds."""
    oj = O.Sim(spec.width, spec.height, xy, spec.sim_seed, spec.disp_lo, spec.disp_hi,
               nthreads=build_threads)
    od = copy.deepcopy(oj)
    oj.nthreads = od.nthreads = threads
    move_s, jfa_s, djfa_s = [], [], []
    for _ in range(steps):
        t0 = time.perf_counter()
        oj.move(), od.move()
        t1 = time.perf_counter()
        oj.jfa_step()
        t2 = time.perf_counter()
        od.djfa_step()
        t3 = time.perf_counter()
        move_s.append(t1 - t0), jfa_s.append(t2 - t1), djfa_s.append(t3 - t2)
    return move_s, jfa_s, djfa_s


def cpu_baseline(args, xy_large=None):
    """The CPU oracle, as it is, timed on this host's cores: per-step JFA and
    dJFA ms of the three single-simulation workloads, with the rows of each
    pass split over every CPU the process may use and single-threaded.
    Bounded sample: the 8192^2 workload's first 3 time steps (all threads;
    the headline value), its first step single-threaded, the 4096^2
    workload's first 3 steps (all threads) and first step (one thread), the
    512^2 workload's 5 steps both ways.  --cpu-full times every listed
    workload's first 3 steps single-threaded too."""
    import oracle as O
    from paper_2209_00117_amd import inputs
    nproc, quota, model = host_cpus()
    threads = max(1, min(nproc, int(quota))) if quota else nproc
    one_steps = 3 if args.cpu_full else 1
    rows, value = [], None
    for name, all_steps, single_steps in (("small", 5, 5), ("single", 3, one_steps),
                                          ("large", 3, one_steps)):
        spec = inputs.WORKLOADS[name]().sims[0]
        xy = xy_large if (name == "large" and xy_large is not None) else spec.positions()
        pj = len(O.schedule(spec.width, spec.height, spec.num_seeds, False))
        pd = len(O.schedule(spec.width, spec.height, spec.num_seeds, True,
                            max(abs(spec.disp_lo), abs(spec.disp_hi))))
        for n_thr, steps in ((threads, all_steps), (1, single_steps)):
            mv, js, ds = oracle_steps(O, spec, xy, threads, n_thr, steps)
            px = spec.width * spec.height
            tot = sum(mv) + sum(js) + sum(ds)
            row = {"workload": name, "threads": n_thr, "steps": steps,
                   "jfa_ms_per_step": 1e3 * float(np.mean(js)),
                   "djfa_ms_per_step": 1e3 * float(np.mean(ds)),
                   "move_ms_per_step": 1e3 * float(np.mean(mv)),
                   "pixel_updates_per_s": steps * px * (pj + pd) / tot}
            rows.append(row)
            print(json.dumps({"cpu_oracle": row}), file=sys.stderr, flush=True)
            if name == "large" and n_thr == threads:
                value = row["pixel_updates_per_s"]
    return {"value": value, "unit": "pixel-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"the 8192x8192 S=2^20 workload's first 3 time steps (move both twins, "
                      f"JFA step, dJFA step; VD_0 untimed), rows of each pass split over "
                      f"{threads} threads; per-workload rows below, single-threaded rows "
                      f"over {one_steps} step(s) of the 4096^2 and 8192^2 workloads",
            "nproc": nproc, "cgroup_cpu_quota": quota, "cpu_model": model,
            "per_workload": rows}


def calibrate(torch, nbytes=512 << 20, reps=20):
    """Plain copy of nbytes between two device buffers: reads nbytes and
    writes nbytes per launch."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    for _ in range(3):
        b.copy_(a)
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s0.record()
    for _ in range(reps):
        b.copy_(a)
    s1.record()
    torch.cuda.synchronize()
    ms = s0.elapsed_time(s1) / reps
    print(json.dumps({"calibration": "device copy", "bytes_read": nbytes, "bytes_written": nbytes,
                      "ms_per_copy": ms, "GBps_read_plus_write": 2 * nbytes / (ms / 1e3) / 1e9}),
          flush=True)


def bench_batched(torch, inputs, V, args):
    """64 simulations of uneven sizes.  Timed three ways on the same GPU,
    each over args.steps time steps (move + step): batched dJFA and batched
    JFA (batched moves, fills and splats, one persistent launch per pass
    level over the members that the batch autotuner keeps together, the
    larger members' passes with their own launches and fused last passes;
    the whole step replayed as a hipGraph), and the same 64 simulations run
    one at a time with plain JFA (per-simulation launches, default kernel
    variants).  Every batched member's map equals its one-at-a-time run bit
    for bit (tests/test_gpu_batch.py)."""
    wl = inputs.batched()
    stream = torch.cuda.current_stream()
    specs = wl.sims
    made = [(s, s.positions()) for s in specs]

    def make():
        return [V.Sim(s.width, s.height, xy, stream=stream, disp_lo=s.disp_lo,
                      disp_hi=s.disp_hi, sim_seed=s.sim_seed) for s, xy in made]

    px = sum(s.width * s.height for s in specs)
    out = {}
    for name, mode in (("batched_djfa", V.STEP_DJFA), ("batched_jfa", V.STEP_JFA)):
        sims = make()
        b = V.Batch(sims, stream=stream)
        if not args.no_tune:
            b.autotune(3)   # untimed: persistent grid and which members run solo
        b.set_graph(not args.no_graph)
        lj, ld, grid = b.info()
        upd = sum(s.width * s.height * (sm.info().passes_djfa if mode == V.STEP_DJFA
                                        else sm.info().passes_jfa)
                  for s, sm in zip(specs, sims))
        for _ in range(args.warmup):
            b.step(mode, True)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for i in range(args.steps):
            b.step(mode, True)
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        lat = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
        total = ev[0].elapsed_time(ev[-1])
        out[name] = {"ms_per_step": total / args.steps, "p50_ms": pct(lat, 50),
                     "p99_ms": pct(lat, 99), "pixel_updates_per_s": upd * args.steps / (total / 1e3),
                     "levels": ld if mode == V.STEP_DJFA else lj, "grid": grid,
                     "graph": not args.no_graph}
        b.close()
        for x in sims:
            x.close()
    # baseline: the same simulations one at a time, plain JFA
    sims = make()
    upd = sum(s.width * s.height * sm.info().passes_jfa for s, sm in zip(specs, sims))
    for _ in range(args.warmup):
        for x in sims:
            x.move_seeds()
            x.jfa_step()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for i in range(args.steps):
        for x in sims:
            x.move_seeds()
            x.jfa_step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    lat = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
    total = ev[0].elapsed_time(ev[-1])
    out["sequential_jfa"] = {"ms_per_step": total / args.steps, "p50_ms": pct(lat, 50),
                             "p99_ms": pct(lat, 99),
                             "pixel_updates_per_s": upd * args.steps / (total / 1e3)}
    for x in sims:
        x.close()
    seq = out["sequential_jfa"]["ms_per_step"]
    line = {"metric": METRIC, "value": out["batched_djfa"]["pixel_updates_per_s"],
            "unit": "pixel-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": out["batched_djfa"]["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "int32",
            "data": "synthetic (uniform random seeds and moves, splitmix64)",
            "config": {"workload": wl.name, "sims": len(specs), "pixels": px},
            **out,
            "speedup_vs_sequential_jfa": {"batched_djfa": seq / out["batched_djfa"]["ms_per_step"],
                                          "batched_jfa": seq / out["batched_jfa"]["ms_per_step"]}}
    print(json.dumps(line), flush=True)


def bench_serving(torch, inputs, V, args):
    """256 resident simulations of mixed sizes; Poisson arrivals of time-step
    requests (move + dJFA) at args.rate per second, uniformly over the
    simulations, for 1 s of warm-up and args.seconds measured.  Latency runs
    from submission to the request's completion on the GPU.  Served twice:
    whole steps and continuous batching (batched ticks, the server's default
    policy).  The same arrival stream is then served one request at a time
    with plain JFA (move + JFA per request, each waited for before the next
    starts)."""
    wl = inputs.serving()
    specs = wl.sims
    stream = torch.cuda.current_stream()
    made = [(s, s.positions()) for s in specs]
    fp = sum((V.footprint_bytes(V.config(s.width, s.height, s.num_seeds)) + 255) // 256 * 256
             for s in specs)
    pool = V.Server.footprint_bytes(len(specs)) + fp + (1 << 20)
    warm = 1.0
    times, targets = inputs.poisson_arrivals(args.rate, warm + args.seconds, len(specs))

    def serve(submit, t_start):
        for at, tgt in zip(times, targets):
            while time.perf_counter() - t_start < at:
                pass
            submit(int(tgt), at)

    def run_server(policy, solo=None):
        sv = V.Server(len(specs), pool, stream=stream)
        sv.set_policy(policy)
        if solo is not None:
            sv.set_solo(solo)
        ids = [sv.add_sim(s.width, s.height, xy, disp_lo=s.disp_lo, disp_hi=s.disp_hi,
                          sim_seed=s.sim_seed) for s, xy in made]
        sv.drain()
        t_start = time.perf_counter()
        reset_done = [False]

        def submit_server(tgt, at):
            if not reset_done[0] and at >= warm:
                sv.stats(reset=True)
                reset_done[0] = True
            sv.submit(ids[tgt], V.STEP_DJFA)

        serve(submit_server, t_start)
        sv.drain()
        st = sv.stats()
        sv.close()
        return {"requests": st["completed"], "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                "mean_ms": st["mean_ms"], "max_ms": st["max_ms"],
                "pixel_updates_per_s": st["pixel_updates"] / st["elapsed_s"],
                "requests_per_s": st["completed"] / st["elapsed_s"], "ticks": st["ticks"],
                "elapsed_s": st["elapsed_s"]}

    # whole steps, then continuous batching (batched ticks, the default policy)
    served = run_server(V.SERVE_STEPS)
    served_passes = run_server(V.SERVE_PASSES)
    solo_sweep = []
    if args.serve_solo_sweep:
        for px in (0, 1024 * 1024, 2048 * 2048, 4096 * 4096 + 1):
            r = run_server(V.SERVE_PASSES, px)
            r["solo_px"] = px
            solo_sweep.append(r)
            print(json.dumps({"serve_solo": px, "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"]}),
                  file=sys.stderr, flush=True)
    px = sum(s.width * s.height for s in specs)

    # one request at a time, plain JFA, same arrivals
    sims = [V.Sim(s.width, s.height, xy, stream=stream, disp_lo=s.disp_lo, disp_hi=s.disp_hi,
                  sim_seed=s.sim_seed) for s, xy in made]
    lat, upd = [], [0]
    t_start = time.perf_counter()

    def submit_plain(tgt, at):
        x = sims[tgt]
        x.move_seeds()
        x.jfa_step()
        torch.cuda.synchronize()
        if at >= warm:
            lat.append((time.perf_counter() - t_start - at) * 1e3)
            upd[0] += x.cfg.width * x.cfg.height * x.info().passes_jfa

    serve(submit_plain, t_start)
    plain_elapsed = time.perf_counter() - t_start - warm
    plain = {"requests": len(lat), "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
             "mean_ms": float(np.mean(lat)) if lat else None,
             "pixel_updates_per_s": upd[0] / plain_elapsed}
    for x in sims:
        x.close()
    line = {"metric": METRIC, "value": served["pixel_updates_per_s"], "unit": "pixel-updates/s",
            "n_gpus": 1, "steps": served["requests"], "warmup": 0,
            "ms_per_step": served["mean_ms"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "int32",
            "data": "synthetic (uniform random seeds and moves, Poisson arrivals, splitmix64)",
            "config": {"workload": wl.name, "sims": len(specs), "pixels": px,
                       "rate_per_s": args.rate, "seconds": args.seconds, "pool_bytes": pool},
            "served_djfa": served, "served_djfa_by_passes": served_passes,
            "one_at_a_time_jfa": plain}
    if solo_sweep:
        line["served_djfa_by_passes_solo_sweep"] = solo_sweep
    print(json.dumps(line), flush=True)


def bench_sweep(torch, V, args, wl, label):
    """JFA+e and dJFA with v leading Von Neumann passes and e extra passes
    (Sec. IV-V: JFA+1/+2 and the VN/Moore mix), v, e in {0, 1, 2}: ms per
    step (default kernel variants, no tuning) and, at the last step, the
    share of pixels equal to JFA+e's map and to plain JFA's map.  All
    simulations follow the same seed trajectory."""
    spec = wl.sims[0]
    W, H = spec.width, spec.height
    xy = spec.positions()
    stream = torch.cuda.current_stream()
    kw = dict(disp_lo=spec.disp_lo, disp_hi=spec.disp_hi, sim_seed=spec.sim_seed, label=label)

    def run(sim, dynamic):
        for _ in range(args.warmup):
            sim.move_seeds()
            sim.djfa_step() if dynamic else sim.jfa_step()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps)]
        torch.cuda.synchronize()
        for i in range(args.steps):
            sim.move_seeds()
            ev[2 * i].record(stream)
            sim.djfa_step() if dynamic else sim.jfa_step()
            ev[2 * i + 1].record(stream)
        torch.cuda.synchronize()
        return float(np.mean([ev[2 * i].elapsed_time(ev[2 * i + 1])
                              for i in range(args.steps)]))

    jfa_maps, jfa_ms = {}, {}
    for e in (0, 1, 2):
        sj = V.Sim(W, H, xy, stream=stream, extra_passes=e, **kw)
        jfa_ms[e] = run(sj, False)
        jfa_maps[e] = sj.read_map()
        sj.close()
    rows = []
    for v in (0, 1, 2):
        for e in (0, 1, 2):
            sd = V.Sim(W, H, xy, stream=stream, vn_passes=v, extra_passes=e, **kw)
            ms = run(sd, True)
            md = sd.read_map()
            info = sd.info()
            sd.close()
            rows.append({"vn_passes": v, "extra_passes": e, "passes_djfa": info.passes_djfa,
                         "djfa_ms": ms, "jfa_extra_ms": jfa_ms[e],
                         "sim_vs_jfa_same_extra": float((md == jfa_maps[e]).mean()),
                         "sim_vs_plain_jfa": float((md == jfa_maps[0]).mean())})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    line = {"metric": METRIC, "value": None, "unit": "pixel-updates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "int32",
            "data": "synthetic (uniform random seeds and moves, splitmix64)",
            "config": {"workload": wl.name, "label": args.label, "mode": "sweep"},
            "sweep": rows}
    print(json.dumps(line), flush=True)


def bench_djfam(torch, V, args, W, H, xy, kw, stream, map_jfa, djfae_ms, jfa_ms):
    """dJFAm (Sec. V-C): a twin with the Manhattan metric and the same seed
    trajectory, stepped as many times as the main twins (tuned, warmed up
    and timed the same way, in a loop of its own), then compared with the
    Euclidean JFA map of the same step."""
    km = dict(kw, metric=V.MANHATTAN)
    sm = V.Sim(W, H, xy, stream=stream, **km)
    if not args.no_tune:
        V.autotune(sm.handle, 3)
    for _ in range(args.warmup):
        sm.move_seeds()
        sm.djfa_step()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    for i in range(args.steps):
        sm.move_seeds()
        ev[i][0].record(stream)
        sm.djfa_step()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    ms = [e[0].elapsed_time(e[1]) for e in ev]
    mm = sm.read_map()
    info = sm.info()
    sm.close()
    t = float(np.mean(ms))
    return {"ms_per_step": t, "p50_ms": pct(ms, 50), "p99_ms": pct(ms, 99),
            "pixel_updates_per_s": W * H * info.passes_djfa / (t / 1e3),
            "speedup_vs_jfa": jfa_ms / t, "speedup_djfae_vs_djfam": djfae_ms / t,
            "similarity_vs_jfa": float((mm == map_jfa).mean())}


def bench_churn(torch, V, args, W, H, xy, kw, stream, djfa_ms):
    """A changing seed set: before each step, a share `args.with_churn` of
    the seeds is removed and as many are inserted at uniform random
    positions (the same script for a JFA and a dJFA twin).  Two tables:
    "full" (num_seeds slots, all present: insertions reuse the slots just
    freed, so each dJFA step also purges their old labels) and "headroom"
    (as many spare slots as a step inserts: insertions take slots freed a
    step earlier, no purge).  Reports the dJFA step time (splat, passes, the
    unclaimed-pixel count and its read-back; the purge where needed), the
    host time of the two seed-set calls, the steps redone as JFA, and the
    similarity to the JFA twin at the last step."""
    S = len(xy)
    n = max(1, int(round(args.with_churn * S)))
    out = {"churn_per_step": n, "plain_djfa_ms_per_step": djfa_ms}
    for mode in ("full", "headroom"):
        rng = np.random.default_rng(17)
        if mode == "headroom":
            extra = np.stack([rng.integers(0, W, n), rng.integers(0, H, n)], 1).astype(np.int32)
            xy0 = np.concatenate([xy, extra])
        else:
            xy0 = xy
        cj = V.Sim(W, H, xy0, stream=stream, **kw)
        cd = V.Sim(W, H, xy0, stream=stream, **kw)
        if mode == "headroom":
            spare = np.arange(S, S + n, dtype=np.int32)
            for sim in (cj, cd):
                sim.remove_seeds(spare)
                sim.jfa_step()
        steps = min(args.steps, 50)
        upd_ms, step_ms, wall_ms = [], [], []
        for i in range(args.warmup + steps):
            present = np.flatnonzero(cd.seed_set()[0])
            gone = rng.choice(present, size=min(n, present.size - 1),
                              replace=False).astype(np.int32)
            new = np.stack([rng.integers(0, W, gone.size), rng.integers(0, H, gone.size)],
                           1).astype(np.int32)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cd.remove_seeds(gone)
            cd.insert_seeds(new)
            t1 = time.perf_counter()
            cj.remove_seeds(gone)
            cj.insert_seeds(new)
            cj.move_seeds(), cd.move_seeds()
            cj.jfa_step()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            e0.record(stream)
            cd.djfa_step()
            e1.record(stream)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            if i >= args.warmup:
                upd_ms.append(1e3 * (t1 - t0))
                step_ms.append(e0.elapsed_time(e1))
                wall_ms.append(1e3 * (t3 - t2))
        sim = float((cj.read_map() == cd.read_map()).mean())
        fallbacks = cd.seed_set()[2]
        cj.close(), cd.close()
        out[mode] = {"steps": steps, "djfa_ms_per_step": float(np.mean(step_ms)),
                     "djfa_wall_ms_per_step": float(np.mean(wall_ms)),
                     "host_update_ms": float(np.mean(upd_ms)), "fallbacks": int(fallbacks),
                     "similarity_vs_jfa": sim}
    return out


def bench_readback(torch, V, args, W, H, xy, kw, stream, passes_djfa):
    """The boundary hands diagrams to the host: dJFA steps (move included)
    each followed by vd_read_map of the whole map, into pinned host memory
    and into ordinary (pageable) memory, timed by the host clock around the
    synchronous calls; and the read-back alone.  PCIe-inclusive figures,
    reported beside the main ones, never as the headline value."""
    sim = V.Sim(W, H, xy, stream=stream, **kw)
    npix = W * H
    pinned = torch.empty(npix, dtype=torch.int32, pin_memory=True)
    pageable = np.empty(npix, np.int32)
    targets = {"pinned": pinned.data_ptr(), "pageable": pageable.ctypes.data}
    steps = min(args.steps, 30)
    out = {"map_bytes": 4 * npix, "steps": steps}
    for name, ptr in targets.items():
        step_ms, copy_ms = [], []
        for i in range(args.warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.move_seeds()
            sim.djfa_step()
            V.read_map_into(sim.handle, ptr, npix)
            t1 = time.perf_counter()
            V.read_map_into(sim.handle, ptr, npix)
            t2 = time.perf_counter()
            if i >= args.warmup:
                step_ms.append(1e3 * (t1 - t0))
                copy_ms.append(1e3 * (t2 - t1))
        ms = float(np.mean(step_ms))
        out[name] = {"djfa_step_with_readback_ms": ms,
                     "readback_ms": float(np.mean(copy_ms)),
                     "readback_GBps": 4 * npix / (float(np.mean(copy_ms)) / 1e3) / 1e9,
                     "pixel_updates_per_s": npix * passes_djfa / (ms / 1e3)}
    sim.close()
    return out


def bench_tail_sweep(torch, V, args):
    """Tail fusion across map sizes: square maps of 256^2 .. 4096^2 with one
    seed per 256 pixels (moves in [-2, 2]), ID and XY labels, the last passes
    of each step separate (0) or fused with 16- or 24-row tiles; ms per JFA
    step and per dJFA step (move included), 40 steps each after 5 warm-up
    steps, default kernel variants."""
    from paper_2209_00117_amd import inputs
    stream = torch.cuda.current_stream()
    rows = []
    for side in (256, 512, 1024, 1536, 2048, 3072, 4096):
        S = max(16, side * side // 256)
        xy = inputs.place_seeds(side, side, S, 3)
        for label in (V.LABEL_ID32, V.LABEL_XY16):
            row = {"side": side, "seeds": S, "label": "id" if label == V.LABEL_ID32 else "xy"}
            for mode in (0, 16, 24):
                sj, sd = (V.Sim(side, side, xy, stream=stream, disp_lo=-2, disp_hi=2, label=label)
                          for _ in range(2))
                for sim in (sj, sd):
                    V.set_tail_fusion(sim.handle, mode)
                for _ in range(5):
                    sj.move_seeds(), sd.move_seeds(), sj.jfa_step(), sd.djfa_step()
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
                torch.cuda.synchronize()
                ev[0].record(stream)
                for _ in range(40):
                    sj.jfa_step()
                ev[1].record(stream)
                for _ in range(40):
                    sd.move_seeds(), sd.djfa_step()
                ev[2].record(stream)
                torch.cuda.synchronize()
                row[f"jfa_ms_{mode}"] = round(ev[0].elapsed_time(ev[1]) / 40, 4)
                row[f"djfa_ms_{mode}"] = round(ev[1].elapsed_time(ev[2]) / 40, 4)
                sj.close(), sd.close()
            print(json.dumps(row), file=sys.stderr, flush=True)
            rows.append(row)
    print(json.dumps({"tail_sweep": rows}), flush=True)


def bench_size_sweep(torch, V, args):
    """Throughput across map sizes: square maps of 1024^2 .. 16368^2 with one
    seed per 256 pixels and moves in [-2, 2], ID and XY labels, each
    autotuned; per size the flood-pass rate of JFA and dJFA steps (HIP events
    around 20 steps of each after 3 warm-up steps) and the share of 8 TB/s
    that the 8 algorithmic bytes per pixel-update make.  The two maps of a
    simulation fit in the 256 MB Infinity Cache up to 4096^2 and not from
    8192^2 on."""
    from paper_2209_00117_amd import inputs
    stream = torch.cuda.current_stream()
    rows = []
    for side in (1024, 2048, 4096, 8192, 11584, 16368):
        S = side * side // 256
        xy = inputs.place_seeds(side, side, S, 7)
        for label in (V.LABEL_ID32, V.LABEL_XY16):
            kw = dict(disp_lo=-2, disp_hi=2, label=label)
            sj = V.Sim(side, side, xy, stream=stream, **kw)
            V.autotune(sj.handle, 2)
            sd = V.Sim(side, side, xy, stream=stream, **kw)
            for _ in range(3):
                sj.move_seeds(), sd.move_seeds(), sj.jfa_step(), sd.djfa_step()
            info = sd.info()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            torch.cuda.synchronize()
            ev[0].record(stream)
            for _ in range(20):
                sj.jfa_step()
            ev[1].record(stream)
            for _ in range(20):
                sd.move_seeds(), sd.djfa_step()
            ev[2].record(stream)
            torch.cuda.synchronize()
            jms, dms = ev[0].elapsed_time(ev[1]) / 20, ev[1].elapsed_time(ev[2]) / 20
            px = side * side
            upd = px * (info.passes_jfa + info.passes_djfa) / ((jms + dms) / 1e3)
            row = {"side": side, "seeds": S, "label": "id" if label == V.LABEL_ID32 else "xy",
                   "map_MiB": 4 * px / 2**20, "passes_jfa": info.passes_jfa,
                   "passes_djfa": info.passes_djfa, "jfa_ms": round(jms, 4),
                   "djfa_ms": round(dms, 4), "G_pixel_updates_per_s": round(upd / 1e9, 1),
                   "hbm_frac_algorithmic": round(8 * upd / 8e12, 3)}
            print(json.dumps(row), file=sys.stderr, flush=True)
            rows.append(row)
            sj.close(), sd.close()
    print(json.dumps({"size_sweep": rows}), flush=True)


def seed_positions_of(labels, name, seeds):
    """(x, y) of each label's seed (int64), and a mask of claimed labels."""
    labels = labels.astype(np.int64)
    if name == "id":
        ok = (labels >= 0) & (labels < len(seeds))
        at = np.where(ok, labels, 0)
        return seeds[at, 0].astype(np.int64), seeds[at, 1].astype(np.int64), ok
    ok = labels >= 0
    return labels & 0xFFFF, labels >> 16, ok


def exact_d2(seeds, px, py):
    """Squared distance from each sample pixel to its exact nearest seed
    (Eq. 1), by a k-d tree over the seeds (scipy); which of several
    equidistant seeds it returns does not matter here."""
    from scipy.spatial import cKDTree
    tree = cKDTree(seeds.astype(np.float64))
    _, idx = tree.query(np.stack([px, py], 1).astype(np.float64), k=1)
    dx = px.astype(np.int64) - seeds[idx, 0]
    dy = py.astype(np.int64) - seeds[idx, 1]
    return dx * dx + dy * dy


def similarity_point(inputs, wl, name, t, seeds, map_jfa, map_djfa):
    """Sec. VI-A similarity at one time step: the share of (sampled) pixels
    whose dJFA (and JFA) label is a seed at exact nearest distance, and the
    paper's dJFA-vs-JFA label equality over the whole map."""
    H, W = map_djfa.shape
    if wl.sample_pixels:
        px, py = inputs.sample_pixels(W, H, wl.sample_pixels, 7)
    else:
        py, px = np.divmod(np.arange(W * H, dtype=np.int64), W)
    px, py = px.astype(np.int64), py.astype(np.int64)
    best = exact_d2(seeds, px, py)
    out = {"t": t}
    for key, m in (("djfa_vs_exact", map_djfa), ("jfa_vs_exact", map_jfa)):
        sx, sy, ok = seed_positions_of(m[py, px], name, seeds)
        d2 = (px - sx) ** 2 + (py - sy) ** 2
        out[key] = float(np.mean(ok & (d2 == best)))
    out["djfa_vs_jfa"] = float((map_djfa == map_jfa).mean())
    out["pixels"] = int(px.size)
    return out


def measure_label(torch, V, args, wl, spec, xy, name):
    """The two twins of one label format on one workload: tuning, warm-up,
    the timed region (the JFA twin's steps, then the dJFA twin's), per-pass
    timing and the similarity checkpoints (t = 1, the end of the timed
    steps, and the workload's full length, all outside the timed region)."""
    from paper_2209_00117_amd import inputs
    W, H = spec.width, spec.height
    label = V.LABEL_ID32 if name == "id" else V.LABEL_XY16
    kw = dict(disp_lo=spec.disp_lo, disp_hi=spec.disp_hi, sim_seed=spec.sim_seed, label=label)
    stream = torch.cuda.current_stream()
    sj = V.Sim(W, H, xy, stream=stream, **kw)
    tuning = None
    if not args.no_tune and not args.load_tuning:
        # Untimed: every pass of both step kinds is timed per kernel variant
        # and segment length on its real input; the twin created next adopts
        # the process-wide table.  The simulation's state is left unchanged.
        V.autotune(sj.handle, 3)
    sd = V.Sim(W, H, xy, stream=stream, **kw)
    if args.tail_fusion != "auto":
        for sim in (sj, sd):
            mode = {"on": 1, "off": 0}.get(args.tail_fusion)
            V.set_tail_fusion(sim.handle, int(args.tail_fusion) if mode is None else mode)
    fused = V.get_tail_fusion(sd.handle)
    info = sd.info()
    pj, pd = info.passes_jfa, info.passes_djfa
    if not args.no_tune:
        ks = [info.k1 >> i for i in range(pj)]
        kd = [info.delta1 >> i for i in range(pd)]
        choice, us = V.get_tuning(sd.handle), V.get_tuning_us(sd.handle)
        rows = [[k, v, r, round(t, 2)] for k, (v, r), t in zip(ks + kd, choice, us)]
        tuning = {"columns": ["k", "variant", "seg_rows", "best_us"], "jfa": rows[:pj],
                  "djfa": rows[pj:], "source": "loaded" if args.load_tuning else "autotuned"}

    def twin_step(sim, dynamic, ev=None):
        # one time step of one twin: its seeds move, then its JFA or dJFA step
        if ev is not None:
            ev[0].record(stream)
        sim.move_seeds()
        if ev is not None:
            ev[1].record(stream)
        sim.djfa_step() if dynamic else sim.jfa_step()
        if ev is not None:
            ev[2].record(stream)

    checks = []

    def checkpoint():
        if args.no_similarity:
            return
        t = sd.info().t
        checks.append(similarity_point(inputs, wl, name, int(t), sd.read_seeds(),
                                       sj.read_map(), sd.read_map()))
        print(json.dumps({"label": name, "similarity": checks[-1]}), file=sys.stderr, flush=True)

    for i in range(args.warmup):
        twin_step(sj, False)
        twin_step(sd, True)
        if i == 0:
            checkpoint()
    torch.cuda.synchronize()

    if not args.no_pass_timing:
        V.set_timing(sj.handle, True)
        V.set_timing(sd.handle, True)
    ev_j, ev_d = ([[torch.cuda.Event(enable_timing=True) for _ in range(3)]
                   for _ in range(args.steps)] for _ in range(2))
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record(stream)
    for i in range(args.steps):
        twin_step(sj, False, ev_j[i])
    for i in range(args.steps):
        twin_step(sd, True, ev_d[i])
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = start.elapsed_time(stop)

    jfa_ms = [e[1].elapsed_time(e[2]) for e in ev_j]
    djfa_ms = [e[1].elapsed_time(e[2]) for e in ev_d]
    move_ms = [a[0].elapsed_time(a[1]) + b[0].elapsed_time(b[1]) for a, b in zip(ev_j, ev_d)]
    tj = tdd = None
    if not args.no_pass_timing:
        tj, tdd = V.get_timing(sj.handle), V.get_timing(sd.handle)
        V.set_timing(sj.handle, False)
        V.set_timing(sd.handle, False)

    # dJFA vs JFA similarity at the last timed step (Sec. VI-A), device maps read back
    mj, md = sj.read_map(), sd.read_map()
    sim_jfa = float((mj == md).mean())
    checkpoint()
    # on to the workload's full length (untimed), then the last checkpoint
    done = args.warmup + args.steps
    if not args.no_similarity and done < spec.steps:
        for _ in range(spec.steps - done):
            twin_step(sj, False)
            twin_step(sd, True)
        checkpoint()

    px_updates = args.steps * W * H * (pj + pd)
    value = px_updates / (total_ms / 1e3)
    roofline = None
    if tj is not None and tj.flood_launches + tdd.flood_launches > 0:
        # per flood pass (the library's pass count; a JFA step's first two
        # passes may share one launch)
        npass = tj.flood_launches + tdd.flood_launches
        avg_ms = (tj.flood_ms + tdd.flood_ms) / npass
        achieved = BYTES_PER_PIXEL_UPDATE * W * H / (avg_ms / 1e3) / 1e9
        traffic = measured_traffic(args.workload + ("" if name == "id" else "-xy"))
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic, "kernel": "flood pass",
                    "avg_pass_us": round(avg_ms * 1e3, 3), "passes": npass,
                    "algorithmic_bytes_per_pass": BYTES_PER_PIXEL_UPDATE * W * H,
                    "jfa_avg_pass_us": round(tj.flood_ms / max(tj.flood_launches, 1) * 1e3, 3),
                    "djfa_avg_pass_us": round(tdd.flood_ms / max(tdd.flood_launches, 1) * 1e3,
                                              3)}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pixel-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (uniform random seeds and moves, splitmix64)",
        "config": {"workload": wl.name, "width": W, "height": H, "seeds": spec.num_seeds,
                   "disp": [spec.disp_lo, spec.disp_hi], "label": name,
                   "passes_jfa": pj, "passes_djfa": pd, "k1": info.k1, "delta1": info.delta1,
                   "fused_tail_passes": {"jfa": fused[0], "djfa": fused[1]}},
        "jfa": {"ms_per_step": float(np.mean(jfa_ms)), "p50_ms": pct(jfa_ms, 50),
                "p99_ms": pct(jfa_ms, 99),
                "pixel_updates_per_s": W * H * pj / (np.mean(jfa_ms) / 1e3)},
        "djfa": {"ms_per_step": float(np.mean(djfa_ms)), "p50_ms": pct(djfa_ms, 50),
                 "p99_ms": pct(djfa_ms, 99),
                 "pixel_updates_per_s": W * H * pd / (np.mean(djfa_ms) / 1e3)},
        "move_ms_per_step": float(np.mean(move_ms)),
        "speedup_djfa_vs_jfa": float(np.mean(jfa_ms) / np.mean(djfa_ms)),
        "similarity_djfa_vs_jfa": sim_jfa,
        "similarity_exact": checks,
        "wall_s": wall,
        "roofline": roofline,
        "cpu_baseline": None,
        "tuning": tuning,
    }
    if args.with_djfam:
        out["djfam"] = bench_djfam(torch, V, args, W, H, xy, kw, stream, mj,
                                   float(np.mean(djfa_ms)), float(np.mean(jfa_ms)))
    if args.with_churn > 0:
        out["churn"] = bench_churn(torch, V, args, W, H, xy, kw, stream, float(np.mean(djfa_ms)))
    if args.with_readback:
        out["readback"] = bench_readback(torch, V, args, W, H, xy, kw, stream, pd)
    sj.close(), sd.close()
    return out


def similarity_run(torch, V, wl, name):
    """One workload at its full length with default kernels, both twins;
    similarity to the exact diagram at the first, middle and last steps
    (every step of a workload of at most 5 steps)."""
    from paper_2209_00117_amd import inputs
    spec = wl.sims[0]
    xy = spec.positions()
    label = V.LABEL_ID32 if name == "id" else V.LABEL_XY16
    stream = torch.cuda.current_stream()
    kw = dict(disp_lo=spec.disp_lo, disp_hi=spec.disp_hi, sim_seed=spec.sim_seed, label=label)
    sj, sd = (V.Sim(spec.width, spec.height, xy, stream=stream, **kw) for _ in range(2))
    at = set(range(1, spec.steps + 1)) if spec.steps <= 5 else {1, spec.steps // 2, spec.steps}
    points = []
    for t in range(1, spec.steps + 1):
        sj.move_seeds(), sd.move_seeds()
        sj.jfa_step(), sd.djfa_step()
        if t in at:
            points.append(similarity_point(inputs, wl, name, t, sd.read_seeds(), sj.read_map(),
                                           sd.read_map()))
    sj.close(), sd.close()
    res = {"workload": wl.name, "label": name, "steps": spec.steps, "points": points}
    for key in ("djfa_vs_exact", "jfa_vs_exact", "djfa_vs_jfa"):
        res[key + "_mean"] = float(np.mean([p[key] for p in points]))
        res[key + "_min"] = float(np.min([p[key] for p in points]))
    print(json.dumps({"similarity_run": res}), file=sys.stderr, flush=True)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="large",
                    choices=["small", "single", "large", "band", "batched", "serving"])
    ap.add_argument("--rate", type=float, default=2000.0, help="serving: requests per second")
    ap.add_argument("--seconds", type=float, default=10.0, help="serving: measured seconds")
    ap.add_argument("--serve-solo-sweep", action="store_true",
                    help="serving: batched ticks with several solo thresholds as well")
    ap.add_argument("--no-graph", action="store_true", help="batched: launch kernels directly")
    ap.add_argument("--label", default="both", choices=["id", "xy", "both"],
                    help="label format; both: measure each, report the faster")
    ap.add_argument("--cpu-full", action="store_true",
                    help="CPU oracle: first 3 steps single-threaded as well")
    ap.add_argument("--no-similarity", action="store_true",
                    help="skip the similarity checkpoints against the exact diagram")
    ap.add_argument("--no-similarity-configs", action="store_true",
                    help="skip the 512^2 and 4096^2 similarity runs")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-pass-timing", action="store_true")
    ap.add_argument("--with-djfam", action="store_true",
                    help="also time a Manhattan dJFA twin (dJFAm, Sec. V-C) after the main "
                         "loop and report T_dJFAe/T_dJFAm and its similarity to JFA")
    ap.add_argument("--with-churn", type=float, default=0.0, metavar="FRACTION",
                    help="also time dJFA steps after removing and inserting FRACTION of the "
                         "seeds before each step (a changing seed set)")
    ap.add_argument("--with-readback", action="store_true",
                    help="also time dJFA steps each followed by reading the map back to the "
                         "host (pinned and pageable memory): PCIe-inclusive figures")
    ap.add_argument("--sweep", action="store_true",
                    help="time dJFA for vn_passes in {0,1,2} x extra_passes in {0,1,2} (and "
                         "JFA+extra) on the workload, with similarities to JFA")
    ap.add_argument("--tail-fusion", default="auto",
                    choices=["auto", "on", "off", "16", "24", "32"],
                    help="run each step's last passes (k = 4, 2, 1) as one LDS-tiled launch "
                         "(16, 24, 32: the tile height; on: 16); auto = the default or the "
                         "autotuner's choice")
    ap.add_argument("--size-sweep", action="store_true",
                    help="pixel-update rate of JFA and dJFA steps on square maps of 1024^2 .. "
                         "16368^2 (one seed per 256 pixels), ID and XY labels, autotuned")
    ap.add_argument("--tail-sweep", action="store_true",
                    help="time steps with the last passes separate and fused (16- and 24-row "
                         "tiles) on square maps of 256^2 .. 4096^2, ID and XY labels")
    ap.add_argument("--save-tuning", metavar="PATH",
                    help="write the process-wide tuning table (JSON) after autotuning")
    ap.add_argument("--load-tuning", metavar="PATH",
                    help="adopt a saved tuning table instead of autotuning (profiled runs: "
                         "counter collection distorts the timings the tuner compares)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (run every pass with the default kernel variant)")
    ap.add_argument("--calibrate", action="store_true",
                    help="time a plain device-to-device copy of known size instead (HBM "
                         "reference for the roofline and for scaling rocprof byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (this path has no multi-GPU mode); "
              f"got --gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2209_00117_amd import inputs, vdflood as V

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate:
        calibrate(torch)
        return
    V.lib()
    if args.tail_sweep:
        bench_tail_sweep(torch, V, args)
        return
    if args.size_sweep:
        bench_size_sweep(torch, V, args)
        return
    if args.workload == "batched":
        bench_batched(torch, inputs, V, args)
        return
    if args.workload == "serving":
        bench_serving(torch, inputs, V, args)
        return
    wl = inputs.WORKLOADS[args.workload]()
    spec = wl.sims[0]
    if args.sweep:
        bench_sweep(torch, V, args, wl, V.LABEL_ID32 if args.label == "id" else V.LABEL_XY16)
        return
    xy = spec.positions()
    if args.load_tuning:
        # a table saved by an earlier run: its choices are adopted by the
        # simulations created below, and nothing is timed here
        V.load_tuning(args.load_tuning)
    names = ["id", "xy"] if args.label == "both" else [args.label]
    results = {name: measure_label(torch, V, args, wl, spec, xy, name) for name in names}
    if args.save_tuning and not args.load_tuning and not args.no_tune:
        V.save_tuning(args.save_tuning)
    # the label format is chosen by measurement: the line reports the faster one
    chosen = max(names, key=lambda n: results[n]["value"])
    out = dict(results[chosen])
    out["config"] = dict(out["config"], label=chosen,
                         label_choice="measured: the faster of " + " and ".join(names))
    if len(names) > 1:
        out["labels"] = {n: {k: results[n][k] for k in
                             ("value", "ms_per_step", "jfa", "djfa", "move_ms_per_step",
                              "speedup_djfa_vs_jfa", "similarity_djfa_vs_jfa",
                              "similarity_exact", "roofline", "tuning")}
                         for n in names}
    if not args.no_similarity_configs and args.workload == "large":
        # dJFA similarity against the exact diagram per workload (Sec. VI-A):
        # the two smaller workloads at their full lengths, default kernels
        out["similarity_per_config"] = [
            similarity_run(torch, V, inputs.WORKLOADS[w](), n)
            for w in ("small", "single") for n in names]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args, xy if args.workload == "large" else None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
