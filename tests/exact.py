"""Independent reference quantities used to pin the oracle.

Nothing here calls the oracle.  It holds:
  - exact enumeration of small periodic lattices with the forward-bond
    Hamiltonian H = -J sum_i sum_{d<dim} s_i s_{i+e_d} (paper Eq. 2);
  - Onsager's internal energy and Yang's spontaneous magnetisation of the
    infinite square-lattice Ising model (textbook closed forms, k_B = J = 1);
  - a blocking estimate of the standard error of a correlated series.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def _forward_bonds(s: np.ndarray, axes) -> np.ndarray:
    """sum_i sum_d s_i s_{i+e_d} for a batch of lattices (batch axis 0)."""
    tot = np.zeros(s.shape[0], dtype=np.int64)
    for ax in axes:
        tot += np.sum(s.astype(np.int64) * np.roll(s, -1, axis=ax), axis=tuple(range(1, s.ndim)))
    return tot


def enumerate_spin_half(shape):
    """All 2^N configurations of +-1 spins: (bond_sum, mag) arrays."""
    n = int(np.prod(shape))
    idx = np.arange(2 ** n, dtype=np.int64)
    bits = ((idx[:, None] >> np.arange(n)) & 1).astype(np.int8)
    s = (1 - 2 * bits).reshape((-1,) + tuple(shape))
    axes = list(range(1, len(shape) + 1))
    return _forward_bonds(s, axes), s.reshape(len(idx), -1).sum(axis=1).astype(np.int64)


def enumerate_spin_one_4x4():
    """Density of states g(bond_sum, mag) of the 4x4 periodic spin-1 lattice,
    built row by row: 81 row states, rows 0..3 with periodic closure."""
    rows = np.array(list(itertools.product((-1, 0, 1), repeat=4)), dtype=np.int64)  # (81, 4)
    e_row = np.sum(rows * np.roll(rows, -1, axis=1), axis=1)  # horizontal bonds of a row
    m_row = rows.sum(axis=1)
    v = rows @ rows.T  # vertical bonds between consecutive rows (81, 81)
    B0, M0 = 32, 16  # offsets: |bond| <= 32, |mag| <= 16
    g = np.zeros((65, 33), dtype=np.int64)
    r2 = np.arange(81)[:, None]
    r3 = np.arange(81)[None, :]
    for r0 in range(81):
        for r1 in range(81):
            b = (e_row[r0] + e_row[r1] + e_row[r2] + e_row[r3]
                 + v[r0, r1] + v[r1, r2] + v[r2, r3] + v[r3, r0])
            m = m_row[r0] + m_row[r1] + m_row[r2] + m_row[r3]
            np.add.at(g, (b + B0, m + M0), 1)
    bonds, mags = np.nonzero(g)
    return bonds - B0, mags - M0, g[bonds, mags]


def canonical_averages(bond, mag, T, N, weight=None, J=1.0):
    """Exact <e>, <|m|>, <m^2> per site and C/N at temperature T."""
    bond = np.asarray(bond, dtype=np.float64)
    mag = np.asarray(mag, dtype=np.float64)
    w = np.ones_like(bond) if weight is None else np.asarray(weight, dtype=np.float64)
    E = -J * bond
    lw = np.log(w) - E / T
    lw -= lw.max()
    p = np.exp(lw)
    p /= p.sum()
    e = float(np.sum(p * E) / N)
    e2 = float(np.sum(p * E * E))
    am = float(np.sum(p * np.abs(mag)) / N)
    m2 = float(np.sum(p * mag * mag) / N ** 2)
    c = (e2 - (e * N) ** 2) / (N * T * T)
    return e, am, m2, c


def onsager_energy(T: float) -> float:
    """Internal energy per site of the infinite 2D Ising model (Onsager 1944)."""
    from scipy.special import ellipk

    b = 1.0 / T
    k = 2.0 * math.sinh(2 * b) / math.cosh(2 * b) ** 2
    K1 = float(ellipk(k * k))
    return -(1.0 / math.tanh(2 * b)) * (1.0 + (2.0 / math.pi) * (2.0 * math.tanh(2 * b) ** 2 - 1.0) * K1)


def yang_magnetisation(T: float) -> float:
    """Spontaneous magnetisation per site below T_c (Yang 1952); 0 above."""
    s = math.sinh(2.0 / T)
    x = 1.0 - s ** -4
    return x ** 0.125 if x > 0 else 0.0


def blocked_mean_err(x: np.ndarray, nblocks: int = 50):
    """Mean and standard error from nblocks contiguous blocks."""
    x = np.asarray(x, dtype=np.float64)
    n = (len(x) // nblocks) * nblocks
    blocks = x[:n].reshape(nblocks, -1).mean(axis=1)
    return float(blocks.mean()), float(blocks.std(ddof=1) / math.sqrt(nblocks))


def _log2cosh(x: float) -> float:
    ax = abs(x)
    return ax + math.log1p(math.exp(-2.0 * ax)) if ax > 0 else math.log(2.0)


def _log2sinh(x: float):
    """(log |2 sinh x|, sign of sinh x)."""
    if x == 0.0:
        return -math.inf, 0.0
    ax = abs(x)
    return ax + math.log1p(-math.exp(-2.0 * ax)), math.copysign(1.0, x)


def kaufman_log_z(L: int, K: float) -> float:
    """log Z of the L x L periodic square-lattice Ising model with coupling K = J/T
    and H = -J sum over the 2 L^2 nearest-neighbour bonds (Kaufman 1949, in the form of
    Ferdinand & Fisher 1969): Z = 1/2 (2 sinh 2K)^{L^2/2} (Z1 + Z2 + Z3 + Z4) with
    Z1,2 = prod_r 2 cosh / 2 sinh (L g_{2r+1} / 2), Z3,4 the same over g_{2r},
    cosh g_l = cosh 2K coth 2K - cos(pi l / L) and g_0 = 2K + ln tanh K (signed)."""
    m = n = L
    c2, s2 = math.cosh(2 * K), math.sinh(2 * K)

    def gamma(l):
        if l == 0:
            return 2 * K + math.log(math.tanh(K))
        return math.acosh(c2 * c2 / s2 - math.cos(math.pi * l / n))

    odd = [gamma(2 * r + 1) for r in range(n)]
    even = [gamma(2 * r) for r in range(n)]
    terms = []  # (log |Z_i|, sign)
    terms.append((sum(_log2cosh(m * g / 2) for g in odd), 1.0))
    ls, sg = 0.0, 1.0
    for g in odd:
        a, b = _log2sinh(m * g / 2)
        ls, sg = ls + a, sg * b
    terms.append((ls, sg))
    terms.append((sum(_log2cosh(m * g / 2) for g in even), 1.0))
    ls, sg = 0.0, 1.0
    for g in even:
        a, b = _log2sinh(m * g / 2)
        ls, sg = ls + a, sg * b
    terms.append((ls, sg))
    top = max(t[0] for t in terms if t[1] != 0.0)
    acc = sum(sg * math.exp(lg - top) for lg, sg in terms if sg != 0.0)
    return math.log(0.5) + 0.5 * m * n * math.log(2 * s2) + top + math.log(acc)


def kaufman_energy_heat(L: int, T: float, h: float = 1e-3):
    """Exact finite-L energy per site <e> and heat capacity per site C/N at T
    (J = 1), by central differences of log Z in K = 1/T."""
    K = 1.0 / T
    f0 = kaufman_log_z(L, K)
    fp, fm = kaufman_log_z(L, K + h), kaufman_log_z(L, K - h)
    fpp, fmm = kaufman_log_z(L, K + 2 * h), kaufman_log_z(L, K - 2 * h)
    d1 = (8 * (fp - fm) - (fpp - fmm)) / (12 * h)
    d2 = (16 * (fp + fm) - (fpp + fmm) - 30 * f0) / (12 * h * h)
    N = L * L
    return -d1 / N, K * K * d2 / N
