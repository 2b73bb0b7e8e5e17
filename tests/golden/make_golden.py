"""Write the full-length golden hashes of the benchmarked configurations.

Runs the CPU oracle (and nothing else) over each configuration at its stated
length and stores, at regular checkpoints, the SHA-256 of the lattice (natural
row-major int8 bytes, NE bytes with the flag bit) and the SHA-256 of the
record series r_0 .. r_n (rows {t, bond_sum, mag, accepted, unflipped} as
little-endian int64).  The GPU test ``tests/test_gpu_full_length.py`` runs
the same configurations through the C ABI and compares both hashes at every
checkpoint.

Configurations (the paper's workloads: 2D Ising on square lattices, Sec. 3.1
and 5.1; 3D and spin-1 as the extension Sec. 3 allows; the North-East model
below c* ~ 0.3, Sec. 3.2 and 5.2), seed 1 everywhere:
  - 2D spin-1/2 Ising 64^2, cold start, T = 2.269, 1000 sweeps;
  - 2D spin-1/2 Ising 8192^2, random start, T in {2.0, 2.269, 2.6}, 10^4 sweeps;
  - 3D Ising 256^3, random start, spin-1/2 at T = 4.5115 and spin-1 at T = 3.19
    (critical estimates), 5000 sweeps;
  - 2D North-East 4096^2, Bernoulli(c) start, c in {0.05, 0.1, 0.2}, 10^5 sweeps.

Usage (from the repository root; hours of CPU for the large cases):
  python tests/golden/make_golden.py [--only CASE ...] [--threads N] [--state-dir DIR]
A file is rewritten after every checkpoint, so an interrupted run leaves a
valid prefix.  With --state-dir the lattice and records are saved there at each
checkpoint and a later run resumes from them.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402

# name -> (oracle parameters, total sweeps, checkpoint interval)
CASES = {
    "ising2d_L64_cold_T2.269": (dict(model=O.ISING, dim=2, L=64, T=2.269, init=O.INIT_COLD), 1000, 100),
    "ising3d_L256_s12_T4.5115": (dict(model=O.ISING, dim=3, L=256, T=4.5115), 5000, 500),
    "ising3d_L256_s1_T3.19": (dict(model=O.ISING, dim=3, L=256, two_s=2, T=3.19), 5000, 500),
    "ne2d_L4096_c0.1": (dict(model=O.NORTH_EAST, dim=2, L=4096, c=0.1), 100000, 10000),
    "ising2d_L8192_T2.269": (dict(model=O.ISING, dim=2, L=8192, T=2.269), 10000, 1000),
    "ne2d_L4096_c0.05": (dict(model=O.NORTH_EAST, dim=2, L=4096, c=0.05), 100000, 10000),
    "ne2d_L4096_c0.2": (dict(model=O.NORTH_EAST, dim=2, L=4096, c=0.2), 100000, 10000),
    "ising2d_L8192_T2.0": (dict(model=O.ISING, dim=2, L=8192, T=2.0), 10000, 1000),
    "ising2d_L8192_T2.6": (dict(model=O.ISING, dim=2, L=8192, T=2.6), 10000, 1000),
}

MODEL_NAMES = {O.ISING: "ising", O.NORTH_EAST: "north_east"}


def params_of(kw) -> O.Params:
    return O.Params(seed=1, **kw)


def describe(p: O.Params) -> dict:
    return {"model": MODEL_NAMES[p.model], "dim": p.dim, "L": p.L, "two_s": p.two_s,
            "J": p.J, "h": p.h, "T": p.T, "c": p.c, "seed": p.seed,
            "init": "cold" if p.init == O.INIT_COLD else "random", "t0": 0}


def run_case(name: str, threads: int, state_dir: str | None) -> None:
    kw, total, every = CASES[name]
    p = params_of(kw)
    out_path = os.path.join(HERE, f"{name}.json")
    s = O.init_lattice(p)
    recs = [O.initial_record(p, s)[None, :]]
    done = 0
    checkpoints = []
    if state_dir:
        st = os.path.join(state_dir, name)
        if os.path.exists(st + ".json"):
            meta = json.load(open(st + ".json"))
            s = np.load(st + "_lattice.npy")
            recs = [np.load(st + "_records.npy")]
            done = meta["done"]
            checkpoints = meta["checkpoints"]
            print(f"{name}: resuming at sweep {done}", flush=True)
    while done < total:
        n = min(every, total - done)
        t0 = time.perf_counter()
        recs.append(O.run(p, s, done, n, records=True, nthreads=threads))
        done += n
        allrec = np.ascontiguousarray(np.vstack(recs), dtype="<i8")
        recs = [allrec]
        checkpoints.append({
            "sweeps": done,
            "lattice_sha256": hashlib.sha256(np.ascontiguousarray(s).tobytes()).hexdigest(),
            "records_sha256": hashlib.sha256(allrec.tobytes()).hexdigest(),
            "last_record": [int(v) for v in allrec[-1]],
        })
        doc = {
            "case": name,
            "what": "SHA-256 of the oracle's lattice and record series r_0..r_n after n sweeps",
            "params": describe(p),
            "sweeps": total,
            "lattice_bytes": "natural row-major int8 [z][y][x] (NE: n | flag << 1)",
            "records_layout": "rows {t, bond_sum, mag, accepted, unflipped}, little-endian int64, r_0 first",
            "generator": "tests/golden/make_golden.py (calls only oracle/)",
            "checkpoints": checkpoints,
        }
        tmp = out_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(doc, fh, indent=1)
            fh.write("\n")
        os.replace(tmp, out_path)
        if state_dir:
            os.makedirs(state_dir, exist_ok=True)
            st = os.path.join(state_dir, name)
            np.save(st + "_lattice.npy", s)
            np.save(st + "_records.npy", allrec)
            with open(st + ".json", "w") as fh:
                json.dump({"done": done, "checkpoints": checkpoints}, fh)
        print(f"{name}: {done}/{total} sweeps ({(time.perf_counter() - t0) / n:.3f} s/sweep)", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", default=None, help="cases to run (default: all, in order)")
    ap.add_argument("--threads", type=int, default=0, help="oracle threads (0: OpenMP default)")
    ap.add_argument("--state-dir", default=None, help="save/resume lattice state here")
    args = ap.parse_args()
    names = args.only or list(CASES)
    for n in names:
        if n not in CASES:
            raise SystemExit(f"unknown case {n}; known: {', '.join(CASES)}")
    for n in names:
        run_case(n, args.threads, args.state_dir)


if __name__ == "__main__":
    main()
