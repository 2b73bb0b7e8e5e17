"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

Holds the workload shapes only (sizes, temperatures, seeds, starts) and a
seeded generator of natural-order lattices for the buffer-initialised path;
none of the method's arithmetic lives here.  Shapes follow the paper's runs
(2D Ising on square lattices, Sec. 3.1 and 5.1; the North-East model at
concentrations below c* ~ 0.3, Sec. 3.2 and 5.2) at the sizes of the
benchmarked configurations.
"""
from __future__ import annotations

import math

import numpy as np

TC_2D = 2.0 / math.log(1.0 + math.sqrt(2.0))  # exact 2D Ising critical temperature

# name -> keyword arguments of Params (model 0 = Ising, 1 = North-East by
# checkerboard, 2 = North-East by random sub-lattices, 3 = its balanced variant,
# 4 = North-East constraint on the Ising energy)
CONFIGS = {
    # 64x64, cold start, T = 2.269, 1000 sweeps, records every sweep
    "ising2d_L64": dict(model=0, dim=2, L=64, two_s=1, J=1.0, h=0.0, T=2.269, seed=1, init=0,
                        sweeps=1000),
    # 8192x8192, random +-1 start, T in {2.0, 2.269, 2.6}, 10^4 sweeps
    "ising2d_L8192": dict(model=0, dim=2, L=8192, two_s=1, J=1.0, h=0.0, T=2.269, seed=1, init=1,
                          sweeps=10000, temperatures=(2.0, 2.269, 2.6)),
    # 32768x32768 (1 GiB per lattice copy, beyond the 256 MB last-level cache): the
    # same sweep measured against HBM itself
    "ising2d_L32768": dict(model=0, dim=2, L=32768, two_s=1, J=1.0, h=0.0, T=2.269, seed=1, init=1,
                           sweeps=1000),
    # 256^3 spin-1/2 and spin-1, random start, T = 0.9..1.1 x critical estimate, 5000 sweeps
    "ising3d_L256_s12": dict(model=0, dim=3, L=256, two_s=1, J=1.0, h=0.0, T=4.5115, seed=1,
                             init=1, sweeps=5000),
    "ising3d_L256_s1": dict(model=0, dim=3, L=256, two_s=2, J=1.0, h=0.0, T=3.19, seed=1, init=1,
                            sweeps=5000),
    # North-East 4096x4096, Bernoulli(c) start, c in {0.05, 0.1, 0.2}, 10^5 sweeps
    "ne2d_L4096": dict(model=1, dim=2, L=4096, two_s=1, c=0.1, seed=1, init=1, sweeps=100000,
                       concentrations=(0.05, 0.1, 0.2)),
    # the same lattice by the paper's random sub-lattice algorithm: 32x32
    # sub-lattices, lambda = 16 (the paper's best setting, Fig. 5)
    "ne2d_sub_L4096": dict(model=2, dim=2, L=4096, two_s=1, c=0.1, seed=1, init=1, sweeps=100000,
                           ne_side=32, ne_lambda=16),
    # its balanced variant (colour 0, then colour 1 sites; four launches per sweep)
    "ne2d_subbal_L4096": dict(model=3, dim=2, L=4096, two_s=1, c=0.1, seed=1, init=1,
                              sweeps=100000, ne_side=32, ne_lambda=16),
    # the NE constraint on the Ising energy (J = 1, h = 0, T = 3), Bernoulli(1/2) start
    "ne2d_coupled_L4096": dict(model=4, dim=2, L=4096, two_s=1, J=1.0, h=0.0, T=3.0, c=0.5,
                               seed=1, init=1, sweeps=100000),
}

# critical-temperature estimates used only to place temperatures (results do
# not depend on them): 3D spin-1/2 and 3D spin-1 simple-cubic Ising
TC_ESTIMATE = {(3, 1): 4.5115, (3, 2): 3.19, (2, 1): TC_2D, (2, 2): 1.6935}


def ne_temperature(c: float) -> float:
    """T for NE up-density c = 1/(1+e^{1/T})."""
    return 1.0 / math.log((1.0 - c) / c)


def random_lattice(shape, two_s: int = 1, seed: int = 0, model: int = 0,
                   flag_fraction: float = 0.0) -> np.ndarray:
    """Seeded natural-order int8 lattice: Ising values in {-1,+1} or {-1,0,+1};
    NE bytes n | flag << 1 with n ~ Bernoulli(1/2) and flags set at random."""
    rng = np.random.default_rng(seed)
    if model != 0:  # every North-East model stores n | flag << 1
        n = rng.integers(0, 2, size=shape, dtype=np.int8)
        f = (rng.random(size=shape) < flag_fraction).astype(np.int8)
        return (n | (f << 1)).astype(np.int8)
    if two_s == 1:
        return (2 * rng.integers(0, 2, size=shape, dtype=np.int8) - 1).astype(np.int8)
    return rng.integers(-1, 2, size=shape, dtype=np.int8)


def served_requests(n: int = 4096, rate: float = 1000.0, seed: int = 5,
                    sweeps=(1000, 10000)):
    """Poisson stream of independent Ising jobs shaped like the served batch:
    2D L log-uniform in [32, 1024] or 3D L log-uniform in [16, 128] (rounded to
    a multiple of 8), spin-1/2 or spin-1, T uniform in [0.8, 1.2] x T_c of the
    model, a sweep count uniform in `sweeps`, and a distinct seed per job.
    Returns a list of dicts {id, arrival (s), dim, L, two_s, T, seed, sweeps}."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        dim = 2 if rng.random() < 0.5 else 3
        lo, hi = (32, 1024) if dim == 2 else (16, 128)
        L = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        L = int(min(hi, max(lo, 8 * round(L / 8))))
        two_s = 1 if rng.random() < 0.5 else 2
        T = float(rng.uniform(0.8, 1.2) * TC_ESTIMATE[(dim, two_s)])
        out.append(dict(id=i, arrival=t, dim=dim, L=L, two_s=two_s, T=T, seed=100000 + i,
                        sweeps=int(rng.integers(sweeps[0], sweeps[1] + 1))))
    return out
