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
    for waves in (4, 16):
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
