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
