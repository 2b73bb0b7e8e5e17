"""Shared helpers of the GPU parity tests: run a configuration through the
C ABI (via the binding) and through the oracle, on the same parameters."""
from __future__ import annotations

import numpy as np

import oracle as O
import paper_1209_0296_amd as S


def oracle_params(sp: S.Params) -> O.Params:
    model = {S.ISING: O.ISING, S.NORTH_EAST: O.NORTH_EAST, S.NE_SUBLATTICE: O.NE_TILES,
             S.NE_SUBLATTICE_BALANCED: O.NE_BALANCED, S.NE_COUPLED: O.NE_COUPLED}[sp.model]
    return O.Params(model=model, dim=sp.dim, L=sp.L, two_s=sp.two_s,
                    init=O.INIT_COLD if sp.init == S.INIT_COLD else O.INIT_RANDOM,
                    J=sp.J, h=sp.h, T=sp.T, c=sp.c, seed=sp.seed,
                    tile=sp.ne_side, lam=sp.ne_lambda)


def run_oracle(sp: S.Params, nsweeps: int, start=None, nthreads: int = 0):
    """Oracle lattice after nsweeps and the records r_0..r_n as (n+1, 5) int64."""
    op = oracle_params(sp)
    s = O.init_lattice(op) if start is None else np.ascontiguousarray(start.copy())
    r0 = O.initial_record(op, s, t=sp.t0)
    if op.model == O.ISING:
        r0[4] = -1
    recs = O.run(op, s, sp.t0, nsweeps, nthreads=nthreads)
    return s, np.vstack([r0[None, :], recs])


def run_gpu(sp: S.Params, nsweeps: int, launch=None, chunks=None, init_spins=None):
    """GPU lattice after nsweeps and all records (incl. r_0) as (n+1, 5) int64."""
    import torch

    lat = S.Lattice(sp, init_spins=None if init_spins is None else torch.from_numpy(init_spins))
    if launch is not None:
        lat.set_launch(*launch)
    recs = [S.records_to_array(lat.measure())]
    for n in (chunks or [nsweeps]):
        lat.sweep(n)
        recs.append(S.records_to_array(lat.measure()))
    spins = lat.spins()
    lat.close()
    return spins, np.vstack(recs)


# ---------------------------------------------------------------------------
# Which launch schedules the library must accept for a shape (include/spinlat.h,
# sl_set_launch): a refusal outside these rules, or an acceptance inside a
# refusal, is a failure, never a skip.

RESIDENT_MAX_BYTES = 48 * 1024  # both colours of the lattice in one workgroup's LDS


def _row_fits(sp: S.Params, H: int, D: int, fused: bool) -> bool:
    """Whole-row kernels: a colour row of L/8 words splits into row groups of
    R = L/(8D) lanes, R <= 64 or a multiple of 64 up to 1024; FUSED is 2D."""
    if D not in (1, 2, 4) or H < 1 or (fused and sp.dim != 2):
        return False
    ncols = sp.L // 8
    if ncols % D:
        return False
    R = ncols // D
    return R <= 64 or (R % 64 == 0 and R <= 1024)


def expected_supported(sp: S.Params, launch) -> bool:
    mode, H, D = launch
    if sp.model in (S.NE_SUBLATTICE, S.NE_SUBLATTICE_BALANCED):
        return mode == S.MODE_AUTO
    if mode in (S.MODE_AUTO, S.MODE_SIMPLE):
        return True
    if mode == S.MODE_RESIDENT:
        return H == 0 and D == 0 and sp.nsites <= RESIDENT_MAX_BYTES
    spin_half_table = (sp.model == S.ISING and sp.two_s == 1) or sp.model == S.NE_COUPLED
    if mode in (S.MODE_HALF, S.MODE_FUSED):
        if spin_half_table and 0 in S.threshold_table(sp):
            return False  # the 32-bit "word <= thr - 1" table needs every threshold >= 1
        fused = mode == S.MODE_FUSED
        H = H or 8
        if D == 0:
            D = next((d for d in (2, 4, 1) if _row_fits(sp, H, d, fused)), 2)
        return _row_fits(sp, H, D, fused)
    if mode == S.MODE_HALF_ROWS:
        if spin_half_table and 0 in S.threshold_table(sp):
            return False
        if H < 0 or H > 16:
            return False
        ncols = sp.L // 8

        def fits(d):
            # one wave per row group; Ising rows may be ragged: the last lane
            # of at least two holds the row's last d words
            if d not in (1, 2, 4):
                return False
            if ncols % d == 0:
                return ncols // d <= 64
            return sp.model == S.ISING and 2 <= -(-ncols // d) <= 64

        if D == 0:
            D = next((d for d in (4, 2, 1) if fits(d)), 4)
        return fits(D)
    if mode in (S.MODE_HALF_WINDOW, S.MODE_FUSED_WINDOW):
        if sp.model == S.NE_COUPLED:
            return False
        if D != 0 or H < 0 or H > sp.L:
            return False
        return mode == S.MODE_HALF_WINDOW or sp.dim == 2
    raise ValueError(f"unknown mode {mode}")


def assert_refused(sp: S.Params, launch) -> None:
    """The schedule must be refused with SL_E_UNSUPPORTED."""
    lat = S.Lattice(sp)
    try:
        try:
            lat.set_launch(*launch)
        except S.SpinlatError as e:
            assert e.status == 2, e
            return
        raise AssertionError(f"schedule {launch} was accepted for {sp}")
    finally:
        lat.close()
