"""Calibration of lambda for the NE sub-lattice algorithm (paper Sec. 3.2, Fig. 5).

The paper fixes lambda by comparing the spin autocorrelation Phi(t) (Eq. 4)
of the parallel algorithm with a single-block, near-serial reference run:
lambda is acceptable while the curves agree.  Here the reference is one
sub-lattice covering the whole lattice (B = L, so every neighbour is read
live) with lambda = 2, the smallest the kernels take; the candidates use
B x B sub-lattices with the given lambda values.  Every run goes through the
library (sweeps, overlap and Phi on the GPU path); realizations differ only
in their seed.

    python -m paper_1209_0296_amd.calibrate --L 64 --c 0.42 --side 32 \\
        --lambdas 16 64 128 --realizations 30

prints one JSON line with the mean Phi(t) of each setting, its standard error
and the largest deviation from the reference in units of the combined error
(with --others also for the balanced variant and the checkerboard sweep).
"""
from __future__ import annotations

import argparse
import json
import math
from dataclasses import replace

import numpy as np

from .spinlat import NE_SUBLATTICE, NE_SUBLATTICE_BALANCED, NORTH_EAST, Lattice, Params, autocorrelation


def phi_curves(p: Params, times, realizations: int, seed0: int = 1) -> np.ndarray:
    """Phi(t) at the sweep counts `times` (increasing) for `realizations` runs:
    array (realizations, len(times))."""
    out = np.zeros((realizations, len(times)))
    for r in range(realizations):
        q = replace(p, seed=seed0 + r, record_capacity=max(times) + 2)
        lat = Lattice(q)
        ref = lat.copy_spins().clone()
        done = 0
        for k, t in enumerate(times):
            if t > done:
                lat.sweep(t - done)
                lat.measure()
                done = t
            out[r, k] = autocorrelation(q, lat.overlap(ref))
        lat.close()
    return out


def _compare(ref_m, ref_e, cur, realizations):
    m = cur.mean(axis=0)
    e = cur.std(axis=0, ddof=1) / math.sqrt(realizations)
    z = np.abs(m - ref_m) / np.sqrt(e * e + ref_e * ref_e + 1e-300)
    return {"phi": m.tolist(), "err": e.tolist(), "max_z": float(z.max()),
            "max_abs_dev": float(np.abs(m - ref_m).max())}


def calibrate(L: int, c: float, side: int, lambdas, times, realizations: int, seed0: int = 1,
              others: bool = False):
    base = Params(model=NE_SUBLATTICE, dim=2, L=L, c=c)
    ref = phi_curves(replace(base, ne_side=L, ne_lambda=2), times, realizations, seed0)
    ref_m = ref.mean(axis=0)
    ref_e = ref.std(axis=0, ddof=1) / math.sqrt(realizations)
    res = {"L": L, "c": c, "side": side, "realizations": realizations, "times": list(times),
           "reference": {"side": L, "lambda": 2, "phi": ref_m.tolist(), "err": ref_e.tolist()},
           "candidates": []}
    for lam in lambdas:
        cur = phi_curves(replace(base, ne_side=side, ne_lambda=lam), times, realizations,
                         seed0 + 100000)
        res["candidates"].append({"lambda": lam} | _compare(ref_m, ref_e, cur, realizations))
    if others:
        # the balanced variant at the smallest lambda, and the checkerboard sweep
        # (Sec. 3.2: it changes the relaxation)
        lam = min(lambdas)
        cur = phi_curves(replace(base, model=NE_SUBLATTICE_BALANCED, ne_side=side, ne_lambda=lam),
                         times, realizations, seed0 + 200000)
        res["balanced"] = {"lambda": lam} | _compare(ref_m, ref_e, cur, realizations)
        cur = phi_curves(replace(base, model=NORTH_EAST), times, realizations, seed0 + 300000)
        res["checkerboard"] = _compare(ref_m, ref_e, cur, realizations)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, default=64)
    ap.add_argument("--c", type=float, default=0.42)
    ap.add_argument("--side", type=int, default=32)
    ap.add_argument("--lambdas", type=int, nargs="+", default=[16, 64, 128])
    ap.add_argument("--times", type=int, nargs="+", default=[1, 2, 4, 8, 16, 32, 64, 128])
    ap.add_argument("--realizations", type=int, default=30)
    ap.add_argument("--others", action="store_true",
                    help="also the balanced variant and the checkerboard sweep")
    a = ap.parse_args()
    print(json.dumps(calibrate(a.L, a.c, a.side, a.lambdas, a.times, a.realizations,
                               others=a.others)), flush=True)


if __name__ == "__main__":
    main()
