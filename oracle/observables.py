"""Observables of a run, from its records or lattices -- TEST INFRASTRUCTURE ONLY.

Plain numpy in double precision, written from the definitions:
  - energy per site e = E/N with E = -J bond_sum - h mag (Eq. 2 with a field),
    magnetisation per site m = mag/N (coupled NE: the same over s = 2n - 1);
  - heat capacity per site C/N = N Var(e) / T^2 (the paper's Fig. 6 compares
    <m>, <e> and C between CPU and GPU), k_B = 1;
  - susceptibility per site chi = N (<m^2> - <|m|>^2) / T (finite-lattice form);
  - Binder cumulant U4 = 1 - <m^4> / (3 <m^2>^2);
  - overlap sum_i s_i(t) s_i(0) and the NE spin autocorrelation of Eq. 4,
    Phi(t) = (overlap/N - <s>^2) / (1 - <s>^2) with <s> = 2c - 1 and
    s = 2n - 1 for an occupation n.
Averages are plain means over the records given (the caller drops the
equilibration part).  Pinned in tests/test_oracle_observables.py.
"""
from __future__ import annotations

import numpy as np

from . import ISING, NE_COUPLED, Params


def spin_sums(p: Params, records):
    """(sum over forward bonds of s_i s_j, sum of s_i) of each record.

    Ising records hold them directly.  NE records count over the occupations
    n = (s + 1) / 2: with b = sum n_i n_j and M = sum n_i over a 2D lattice of
    N sites and 2N forward bonds, each site in four of them,
    sum s_i s_j = 4b - 8M + 2N and sum s_i = 2M - N."""
    r = np.asarray(records, dtype=np.int64)
    bond = r[:, 1].astype(np.float64)
    mag = r[:, 2].astype(np.float64)
    if p.model == ISING:
        return bond, mag
    N = float(p.nsites)
    return 4.0 * bond - 8.0 * mag + 2.0 * N, 2.0 * mag - N


def statistics(p: Params, records) -> dict:
    """Means and fluctuation observables of an (n, 5) record array of an Ising
    run, or of a coupled NE run in its spin variables."""
    if p.model not in (ISING, NE_COUPLED):
        raise ValueError("thermodynamic statistics are defined for the Ising energy")
    r = np.asarray(records, dtype=np.int64)
    N = float(p.nsites)
    bond, mag = spin_sums(p, r)
    e = (-p.J * bond - p.h * mag) / N
    m = mag / N
    mean_e = float(np.mean(e))
    var_e = float(np.mean((e - mean_e) ** 2))
    m_abs = float(np.mean(np.abs(m)))
    m2 = float(np.mean(m * m))
    m4 = float(np.mean(m ** 4))
    return {
        "n": int(r.shape[0]),
        "e": mean_e,
        "e_var": var_e,
        "m": float(np.mean(m)),
        "m_abs": m_abs,
        "m2": m2,
        "m4": m4,
        "heat_capacity": N * var_e / (p.T * p.T),
        "susceptibility": N * (m2 - m_abs * m_abs) / p.T,
        "binder": 1.0 - m4 / (3.0 * m2 * m2) if m2 > 0 else float("nan"),
    }


def spin_values(p: Params, s: np.ndarray) -> np.ndarray:
    """Spin value of every site: s for Ising, 2n - 1 for the NE occupation n."""
    if p.model == ISING:
        return s.astype(np.int64)
    return 2 * (s.astype(np.int64) & 1) - 1


def overlap(p: Params, s: np.ndarray, ref: np.ndarray) -> int:
    """sum_i s_i s_i^ref over the lattice (natural order arrays)."""
    return int(np.sum(spin_values(p, s) * spin_values(p, ref)))


def autocorrelation(p: Params, ov: int) -> float:
    """NE spin autocorrelation Phi (Eq. 4) from the overlap with the reference."""
    if p.model == ISING:
        raise ValueError("Phi(t) of Eq. 4 is defined for the North-East model")
    m0 = 2.0 * p.c - 1.0
    return (ov / float(p.nsites) - m0 * m0) / (1.0 - m0 * m0)
