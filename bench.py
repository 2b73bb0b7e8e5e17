"""Benchmark of the checkerboard Metropolis sweep on one MI355X.

A step is one full sweep (colour 0 then colour 1, with the fused per-sweep
reduction of bond sum, magnetisation and accepted moves) of the 2D spin-1/2
Ising lattice L = 8192, J = 1, h = 0, T = 2.269, random start from seed 1;
the records of the timed sweeps are drained (measure) inside the timed
region.  The lattice is created and warmed up before timing, so it is
resident in HBM when the timed region starts.

Printed: one JSON line with flip attempts/s, the roofline position of the
sweep kernel (2 algorithmic bytes per attempt: every int8 site read and
written once per sweep), the same for the 3D L = 256 lattice, and the CPU
oracle's rate on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, 8 TB/s
ALGO_BYTES_PER_ATTEMPT = 2   # one int8 read + one int8 write per site per sweep
VALU_WAVE_INSTS_PER_S = 256 * 4 * 2.4e9 / 4  # 3.93e13 32-bit lane-ops/s in wave64 instructions
# sources of the profiled kernels, hashed into profiles/traffic.json
ROW_SOURCES = ("kernels_row.hip", "row_device.hpp", "site_update.hpp", "philox.hpp",
               "spinlat_internal.h", "host_logic.h")
ROWS_SOURCES = ("kernels_rows.hip", "rows_device.hpp", "row_device.hpp", "site_update.hpp", "philox.hpp",
                "spinlat_internal.h", "host_logic.h")
KERNEL_SOURCES = {
    "ising2d_L8192": ROW_SOURCES,
    "ising3d_L256_s12": ROWS_SOURCES,
    "ising3d_L256_s1": ROWS_SOURCES,
    "ne2d_L4096": ROW_SOURCES,
    "ne2d_sub_L4096": ("ne_sub_device.hpp", "philox.hpp", "spinlat_internal.h", "host_logic.h"),
}


def sources_sha256(workload):
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES[workload]:
        with open(os.path.join(ROOT, "paper_1209_0296_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _profile_entry(workload):
    """The committed counter figures of a workload's kernel, or None when the
    kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    entry = json.load(open(path)).get(workload)
    if not entry or sources_sha256(workload) != entry["sources_sha256"]:
        return None
    return entry


def measured_traffic(workload):
    """HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE profile."""
    entry = _profile_entry(workload)
    return entry["bytes_per_launch"] if entry else None


def valu_fraction(workload, per_launch_s):
    """Issued VALU instructions per launch (SQ_INSTS_VALU of the committed
    profile) over what the chip issues in the measured launch time: 256 CUs x
    4 SIMDs, one wave64 instruction per SIMD every 4 cycles at 2.4 GHz."""
    entry = _profile_entry(workload)
    if not entry or "valu_insts_per_dispatch" not in entry:
        return None
    insts = entry["valu_insts_per_dispatch"]
    return {"insts_per_launch": insts, "peak_insts_per_s": VALU_WAVE_INSTS_PER_S,
            "frac": insts / (per_launch_s * VALU_WAVE_INSTS_PER_S)}


def _lattice(S, cfg, T=None, record_capacity=4096):
    p = S.Params(model=cfg["model"], dim=cfg["dim"], L=cfg["L"], two_s=cfg["two_s"],
                 J=cfg.get("J", 1.0), h=cfg.get("h", 0.0), T=T if T is not None else cfg.get("T", 1.0),
                 c=cfg.get("c", 0.1), seed=cfg["seed"], init=cfg["init"],
                 record_capacity=record_capacity, ne_side=cfg.get("ne_side", 32),
                 ne_lambda=cfg.get("ne_lambda", 16))
    return p, S.Lattice(p)


def prewarm(lat, seconds, chunk):
    """Untimed sweeps of the lattice until `seconds` of wall time have passed.
    The GPU clock ramps up only after some tens of ms under load, which a few
    warm-up sweeps of a lattice that takes 20-50 us per sweep do not cover.
    Returns the number of sweeps run."""
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        lat.sweep(chunk)
        lat.measure()
        n += chunk
    return n


def time_workload(S, torch, name, cfg, steps, warmup, T=None, prewarm_s=0.0):
    """Pre-warm, warm up, then time `steps` sweeps plus the drain of their
    records."""
    p, lat = _lattice(S, cfg, T=T, record_capacity=max(steps, warmup, 64) + 2)
    pre = prewarm(lat, prewarm_s, 64) if prewarm_s > 0 else 0
    lat.sweep(warmup)
    lat.measure()
    stream = lat.stream
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    lat.sweep(steps)
    end.record(stream)
    recs = lat.measure()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sweep_ms = start.elapsed_time(end)  # the sweep launches only, on their stream
    assert len(recs) == steps
    mode = lat.get_launch()
    lat.close()
    attempts = p.nsites * steps
    if p.model in (S.NE_SUBLATTICE, S.NE_SUBLATTICE_BALANCED):
        # two (balanced: four) launches per sweep, each reading and writing the lattice
        launches_per_sweep = 2 if p.model == S.NE_SUBLATTICE else 4
        bytes_per_launch = 2 * p.nsites
    else:
        launches_per_sweep = 1 if mode[0] == S.MODE_FUSED else 2
        bytes_per_launch = ALGO_BYTES_PER_ATTEMPT * p.nsites / launches_per_sweep
    per_launch_s = sweep_ms / 1e3 / (steps * launches_per_sweep)
    achieved = bytes_per_launch / per_launch_s / 1e9
    return {
        "workload": name, "attempts_per_s": attempts / wall, "wall_s": wall,
        "ms_per_step": wall * 1e3 / steps, "sweep_kernels_ms_per_step": sweep_ms / steps,
        "launch": {"mode": mode[0], "tile_rows": mode[1], "tile_words": mode[2],
                   "launches_per_sweep": launches_per_sweep},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "per_launch_us": per_launch_s * 1e6, "algo_bytes_per_launch": bytes_per_launch},
        "nsites": p.nsites, "steps": steps, "prewarm_sweeps": pre,
    }


def host_description():
    """What the CPU baseline ran on: core counts, CPU model, oracle build flags."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {"nproc": os.cpu_count(), "affinity_cpus": affinity, "cpu_model": model,
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS"),
            "oracle_build": "gcc -O3 -fno-fast-math -ffp-contract=off -fopenmp (oracle/__init__.py)"}


def baseline_threads():
    """All the host cores this process may use: the OpenMP thread count the
    environment sets for this machine's share, else every CPU in the affinity
    mask."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(cfg, sweeps, threads, single_sweeps=2):
    """The oracle as it is, on the host cores, on `sweeps` sweeps of the same
    lattice; and on one thread over `single_sweeps` sweeps."""
    import oracle as O

    p = O.Params(model=cfg["model"], dim=cfg["dim"], L=cfg["L"], two_s=cfg["two_s"],
                 init=O.INIT_COLD if cfg["init"] == 0 else O.INIT_RANDOM, J=cfg.get("J", 1.0),
                 h=cfg.get("h", 0.0), T=cfg.get("T", 1.0), c=cfg.get("c", 0.1), seed=cfg["seed"])
    s = O.init_lattice(p)
    t0 = time.perf_counter()
    O.run(p, s, 0, sweeps, records=True, nthreads=threads)
    dt = time.perf_counter() - t0
    out = {"value": p.nsites * sweeps / dt, "unit": "flip attempts/s", "cores": threads,
           "kind": "oracle",
           "sample": f"{sweeps} sweeps of 2D L={cfg['L']} (records every sweep), {dt:.1f} s"}
    if single_sweeps:
        t0 = time.perf_counter()
        O.run(p, s, sweeps, single_sweeps, records=True, nthreads=1)
        d1 = time.perf_counter() - t0
        out["single_thread_value"] = p.nsites * single_sweeps / d1
        out["single_thread_sample"] = f"{single_sweeps} further sweeps on 1 thread, {d1:.1f} s"
    out["host"] = host_description()
    return out


def served(args):
    """Continuous batching of a Poisson stream of independent Ising jobs.

    1. The batch autotuner picks the strip height and chunk size on a sample
       of the stream (closed batch).
    2. Capacity: the whole stream as a closed batch (every job waiting at time
       0): jobs/s and attempts/s at saturation.
    3. Latency: the stream offered at 70% of that capacity (Poisson arrivals,
       served in real time): p50/p99 of completion - arrival.
    4. The first `compare_jobs` jobs as a closed batch, batched vs one lattice
       per launch, with identical records; and batched without graph replay."""
    import numpy as np

    from paper_1209_0296_amd import BATCH_NO_GRAPH
    from paper_1209_0296_amd.autotune import autotune_batch
    from paper_1209_0296_amd.serve import Server, requests_from_workload, run_one_per_launch
    from workloads import served_requests

    arena = args.served_arena_mib << 20
    n = args.served_jobs
    say = lambda m: print(f"# served: {m}", file=sys.stderr, flush=True)
    if args.tune_jobs > 0:
        sample = requests_from_workload(served_requests(args.tune_jobs, rate=1e9, seed=7))
        say(f"autotune on {len(sample)} jobs")
        (H, chunk), table = autotune_batch(sample, arena, chunks=(32, 64, 128, 256), log=say)
        say(f"batch autotuner: tile_rows {H}, chunk {chunk} "
            f"({min(table.values()):.3f} s of {max(table.values()):.3f} s)")
    else:
        H, chunk, table = 0, args.served_chunk, {}
    srv = Server(arena, max_jobs=n, chunk=chunk, tile_rows=H)
    closed = requests_from_workload(served_requests(n, rate=1e9))
    attempts = sum(r.params.nsites * r.sweeps for r in closed)
    srv.run(requests_from_workload(served_requests(64, rate=1e9, seed=99, sweeps=(2, 4))), realtime=False)
    say(f"capacity: closed batch of {n} jobs")
    _, cap = srv.run(closed, realtime=False)
    rate = args.served_load * cap["jobs_per_s"]
    stream = requests_from_workload(served_requests(n, rate=rate))
    live = {k: None for k in ("jobs", "jobs_per_s", "p50_latency_s", "p99_latency_s", "makespan_s")}
    if args.served_latency:
        say(f"latency: {n} jobs at {rate:.4g} jobs/s")
        _, live = srv.run(stream, realtime=True)
    out = {"workload": f"served_ising_{n}", "arena_bytes": arena, "tile_rows": H, "chunk_sweeps": chunk,
           "autotune_s": {f"{k[0]},{k[1]}": v for k, v in table.items()},
           "capacity": {"jobs": cap["jobs"], "jobs_per_s": cap["jobs_per_s"], "makespan_s": cap["makespan_s"],
                        "attempts_per_s": attempts / cap["makespan_s"]},
           "offered_load": args.served_load, "arrival_rate_per_s": rate,
           "jobs": live["jobs"], "jobs_per_s": live["jobs_per_s"], "p50_latency_s": live["p50_latency_s"],
           "p99_latency_s": live["p99_latency_s"], "makespan_s": live["makespan_s"],
           "attempts_per_s": attempts / cap["makespan_s"]}
    k = min(args.compare_jobs, n)
    if k:
        sub = closed[:k]
        say(f"compare: {k} jobs batched, without graphs, one per launch")
        o_b, s_b = srv.run(sub, realtime=False)
        srv.close()
        ng = Server(arena, max_jobs=n, chunk=chunk, tile_rows=H, flags=BATCH_NO_GRAPH)
        ng.run(sub[: max(1, k // 8)], realtime=False)
        o_g, s_g = ng.run(sub, realtime=False)
        ng.close()
        o_1, s_1 = run_one_per_launch(sub, realtime=False)
        same = all(np.array_equal(o_b[r.id].records, o_1[r.id].records) and
                   np.array_equal(o_b[r.id].records, o_g[r.id].records) for r in sub)
        out["vs_one_per_launch"] = {"jobs": k, "batched_jobs_per_s": s_b["jobs_per_s"],
                                    "batched_no_graph_jobs_per_s": s_g["jobs_per_s"],
                                    "one_per_launch_jobs_per_s": s_1["jobs_per_s"],
                                    "speedup": s_b["jobs_per_s"] / s_1["jobs_per_s"],
                                    "graph_gain": s_b["jobs_per_s"] / s_g["jobs_per_s"],
                                    "identical_records": bool(same)}
    else:
        srv.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    # the GPU clock takes ~20 ms of load to ramp up: 50 warm-up sweeps of the
    # 2D lattice measured 46.3 us per sweep, 500 measured 43.0 and 2000 42.7
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--prewarm-s", type=float, default=0.2,
                    help="untimed sweeps for this many seconds before the warm-up steps of each "
                         "workload, so that the GPU clock has ramped up (0: none)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 2D L=64 and L=32768, 3D L=256 and NE L=4096 lines")
    ap.add_argument("--cpu-sweeps", type=int, default=100)
    ap.add_argument("--served-jobs", type=int, default=4096,
                    help="jobs in the served Poisson stream (0: skip serving)")
    ap.add_argument("--served-load", type=float, default=0.7,
                    help="offered load of the latency run, as a fraction of the measured capacity")
    ap.add_argument("--served-arena-mib", type=int, default=2048)
    ap.add_argument("--tune-jobs", type=int, default=256,
                    help="sample jobs of the batch autotuner (0: no tuning, default strip "
                         "heights and --served-chunk)")
    ap.add_argument("--served-chunk", type=int, default=256, help="sweeps per chunk without tuning")
    ap.add_argument("--served-latency", type=int, default=1,
                    help="0: skip the run at the offered load (capacity and comparison only)")
    ap.add_argument("--compare-jobs", type=int, default=512,
                    help="jobs served both batched and one run per launch (closed batch)")
    ap.add_argument("--only", default="", metavar="WORKLOAD",
                    help="time only this workload of workloads.CONFIGS and print its own JSON "
                         "line (for profiling one kernel)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (scale for the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU slab decomposition is a design, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n}))
        return

    import paper_1209_0296_amd as S
    from workloads import CONFIGS

    if args.only:
        r = time_workload(S, torch, args.only, CONFIGS[args.only], args.steps, args.warmup,
                          prewarm_s=args.prewarm_s)
        print(json.dumps(r), flush=True)
        return

    cfg2 = CONFIGS["ising2d_L8192"]
    main_res = time_workload(S, torch, "ising2d_L8192_T2.269", cfg2, args.steps, args.warmup,
                             prewarm_s=args.prewarm_s)
    print(f"# 2D L=8192: {main_res['attempts_per_s']:.4g} attempts/s, "
          f"{main_res['ms_per_step']:.4f} ms/sweep", file=sys.stderr, flush=True)
    secondary = []
    if not args.no_secondary:
        for key in ("ising2d_L64", "ising2d_L32768", "ising3d_L256_s12", "ising3d_L256_s1",
                    "ne2d_L4096", "ne2d_sub_L4096", "ne2d_subbal_L4096", "ne2d_coupled_L4096"):
            r = time_workload(S, torch, key, CONFIGS[key], args.steps, args.warmup,
                              prewarm_s=args.prewarm_s)
            print(f"# {key}: {r['attempts_per_s']:.4g} attempts/s, {r['ms_per_step']:.4f} ms/sweep",
                  file=sys.stderr, flush=True)
            per_launch_s = r["roofline"]["per_launch_us"] * 1e-6
            secondary.append({k: r[k] for k in ("workload", "attempts_per_s", "ms_per_step",
                                                 "sweep_kernels_ms_per_step", "launch")}
                             | {"roofline_frac": r["roofline"]["frac"],
                                "per_launch_us": r["roofline"]["per_launch_us"],
                                "algo_bytes_per_launch": r["roofline"]["algo_bytes_per_launch"],
                                # committed counters, while the kernel sources match them
                                "traffic": measured_traffic(key),
                                "valu": valu_fraction(key, per_launch_s)})
    # the served and CPU-baseline sections report an exception in the line
    # instead of losing the headline measurement taken above
    served_res = None
    if args.served_jobs > 0:
        try:
            served_res = served(args)
            print(f"# served: capacity {served_res['capacity']['jobs_per_s']:.4g} jobs/s "
                  f"({served_res['capacity']['attempts_per_s']:.3g} attempts/s); at "
                  f"{served_res['offered_load']:.0%} load p50 {served_res['p50_latency_s']} s, "
                  f"p99 {served_res['p99_latency_s']} s", file=sys.stderr, flush=True)
        except Exception as e:  # noqa: BLE001
            served_res = {"error": f"{type(e).__name__}: {e}"}
            print(f"# served: failed: {served_res['error']}", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu:
        try:
            threads = baseline_threads()
            cpu = cpu_baseline(cfg2, args.cpu_sweeps, threads)
            print(f"# oracle: {cpu['value']:.4g} attempts/s on {threads} threads", file=sys.stderr,
                  flush=True)
        except Exception as e:  # noqa: BLE001
            cpu = {"error": f"{type(e).__name__}: {e}"}
            print(f"# oracle: failed: {cpu['error']}", file=sys.stderr, flush=True)

    roof = dict(main_res["roofline"])
    roof["traffic"] = measured_traffic("ising2d_L8192")
    line = {
        "metric": "flip attempts/s at 2D L=8192 (% HBM peak)",
        "value": main_res["attempts_per_s"],
        "unit": "flip attempts/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "prewarm": {"seconds": args.prewarm_s, "sweeps": main_res["prewarm_sweeps"],
                    "note": "untimed sweeps before the warm-up steps, until the GPU clock has ramped up"},
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "ising2d_L8192_T2.269", "dim": 2, "L": 8192, "spin": "1/2",
                   "J": 1.0, "h": 0.0, "T": 2.269, "start": "random", "seed": 1,
                   "spins": "int8", "launch": main_res["launch"]},
        "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_detail": {"per_launch_us": roof["per_launch_us"],
                            "algo_bytes_per_launch": roof["algo_bytes_per_launch"],
                            "algo_bytes_per_attempt": ALGO_BYTES_PER_ATTEMPT,
                            "valu": valu_fraction("ising2d_L8192", roof["per_launch_us"] * 1e-6)},
        "cpu_baseline": cpu,
        "served": served_res,
        "secondary": secondary,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
