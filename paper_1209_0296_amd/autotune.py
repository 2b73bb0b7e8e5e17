"""Autotuner for the launch schedule of a lattice shape.

Every schedule produces the same lattice and records (the random numbers
depend on seed, sweep and site only), so the choice is a pure speed question.
The tuner times each candidate schedule on a probe lattice of the same shape
and model (its own seed and device buffer; the caller's lattice is never
touched) with HIP events around `sweeps` sweeps after a warm-up, and returns
the fastest together with the timings.  Candidates: the resident mode, the
direct kernel, the whole-row half and fused kernels over strip heights and
words per lane, and the column-window kernels; shapes a schedule does not fit
are skipped.

    best, table = autotune(Params(L=2048, T=2.269))
    lat = Lattice(params); lat.set_launch(*best)
"""
from __future__ import annotations

from dataclasses import replace

from .spinlat import (MODE_FUSED, MODE_FUSED_WINDOW, MODE_HALF, MODE_HALF_ROWS, MODE_HALF_WINDOW, MODE_RESIDENT,
                      MODE_SIMPLE, NE_SUBLATTICE, NE_SUBLATTICE_BALANCED, Lattice, Params,
                      SpinlatError)


def candidates(p: Params):
    out = [(MODE_RESIDENT, 0, 0), (MODE_SIMPLE, 0, 0)]
    modes = (MODE_HALF, MODE_FUSED) if p.dim == 2 else (MODE_HALF,)
    for mode in modes:
        for H in (2, 4, 8, 16):
            for D in (1, 2, 4):
                out.append((mode, H, D))
    for waves in (4, 8, 16):
        for D in (1, 2, 4):
            out.append((MODE_HALF_ROWS, waves, D))
    out.append((MODE_HALF_WINDOW, 0, 0))
    if p.dim == 2:
        out.append((MODE_FUSED_WINDOW, 0, 0))
    return out


def autotune(p: Params, sweeps: int = 0, warmup: int = 0, device="cuda"):
    """Fastest schedule for the shape of `p`: ((mode, tile_rows, tile_words),
    {schedule: seconds per sweep})."""
    import torch

    if p.model in (NE_SUBLATTICE, NE_SUBLATTICE_BALANCED):
        return (0, 0, 0), {}
    if not sweeps:
        sweeps = max(20, min(1000, int(2e9 // max(1, p.nsites))))
    if not warmup:
        warmup = sweeps
    probe = replace(p, seed=p.seed + 0x5EED, record_capacity=max(sweeps, warmup) + 2)
    lat = Lattice(probe, device=device)
    table = {}
    try:
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        for cand in candidates(p):
            try:
                lat.set_launch(*cand)
            except SpinlatError:
                continue
            lat.sweep(warmup)
            lat.measure()
            start.record(lat.stream)
            lat.sweep(sweeps)
            end.record(lat.stream)
            lat.measure()
            table[cand] = start.elapsed_time(end) / 1e3 / sweeps
    finally:
        lat.close()
    best = min(table, key=table.get)
    return best, table


def autotune_batch(requests, arena_bytes: int, tile_rows=(0, 2, 4, 8), chunks=(16, 64, 256),
                   max_jobs: int = 4096, device="cuda", log=None):
    """Fastest batch configuration for a sample of served requests: the strip
    height of the walk and fused classes and the sweeps per chunk, timed as a
    closed batch of `requests` (serve.Request) after one untimed pass of each
    configuration.  Returns ((tile_rows, chunk), {(tile_rows, chunk): seconds}).
    Results do not depend on the choice (every class is bit-identical to the
    lattice run alone).  `log`, if given, is called with one line per
    configuration as it finishes."""
    from .serve import Server

    table = {}
    for H in tile_rows:
        for ch in chunks:
            srv = Server(arena_bytes, max_jobs=max_jobs, chunk=ch, tile_rows=H, device=device)
            try:
                srv.run(requests[: max(1, len(requests) // 8)], realtime=False)  # kernels, graphs
                _, st = srv.run(requests, realtime=False)
            finally:
                srv.close()
            table[(H, ch)] = st["makespan_s"]
            if log:
                log(f"tile_rows {H}, chunk {ch}: {st['makespan_s']:.3f} s")
    best = min(table, key=table.get)
    return best, table
