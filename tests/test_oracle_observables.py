"""Pins of the oracle's observables (oracle/observables.py) and, through them,
of long oracle runs against exact finite-lattice results.

  * heat capacity and Binder cumulant of a record set that samples the exact
    4x4 Boltzmann distribution equal the exact values (heat capacity from the
    second derivative of log Z, not from a variance);
  * a long oracle run on the 64 x 64 lattice reproduces the exact finite-size
    energy and heat capacity of Kaufman's solution (independent of the
    oracle, checked against enumeration at L = 4);
  * Phi(0) = 1 and Phi of independent Bernoulli(c) states vanishes (Eq. 4).
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import observables as OB
from exact import blocked_mean_err, enumerate_spin_half, kaufman_energy_heat, kaufman_log_z


def test_kaufman_matches_enumeration():
    b, _ = enumerate_spin_half((4, 4))
    for T in (1.5, 2.0, 2.269, 2.6, 5.0):
        K = 1.0 / T
        top = (K * b).max()
        lz = math.log(np.sum(np.exp(K * b - top))) + top
        assert abs(lz - kaufman_log_z(4, K)) < 1e-12


@pytest.mark.parametrize("T", [1.8, 2.269, 2.6])
def test_statistics_of_exact_distribution(T):
    """Records drawn in exact proportion to the 4x4 Boltzmann weights (10^6
    pseudo-records); the heat capacity is checked against d^2 log Z / dK^2."""
    b, m = enumerate_spin_half((4, 4))
    K = 1.0 / T
    w = np.exp(K * b - (K * b).max())
    w /= w.sum()
    # aggregate the 2^16 states into (bond, mag) classes, then 2e6 records
    pairs, inv = np.unique(np.stack([b, m], axis=1), axis=0, return_inverse=True)
    pw = np.bincount(inv.ravel(), weights=w)
    cnt = np.round(pw * 2e6).astype(np.int64)
    keep = cnt > 0
    rec = np.zeros((int(cnt.sum()), 5), dtype=np.int64)
    rec[:, 1] = np.repeat(pairs[keep, 0], cnt[keep])
    rec[:, 2] = np.repeat(pairs[keep, 1], cnt[keep])
    p = O.Params(L=4, T=T)
    st = OB.statistics(p, rec)
    e_exact, c_exact = kaufman_energy_heat(4, T)
    assert abs(st["e"] - e_exact) < 1e-4
    assert abs(st["heat_capacity"] - c_exact) < 1e-3 * max(1.0, c_exact)
    # Binder cumulant from the exact moments of m
    m2 = np.sum(w * (m / 16.0) ** 2)
    m4 = np.sum(w * (m / 16.0) ** 4)
    assert abs(st["binder"] - (1 - m4 / (3 * m2 * m2))) < 1e-4
    assert 0.0 <= st["binder"] <= 2.0 / 3.0 + 1e-12


def test_binder_limits():
    """U4 -> 2/3 for an ordered state (m = +-1) and 0 for a Gaussian m."""
    p = O.Params(L=8, T=1.0)
    rec = np.zeros((1000, 5), dtype=np.int64)
    rec[:, 2] = np.where(np.arange(1000) % 2 == 0, 64, -64)
    assert abs(OB.statistics(p, rec)["binder"] - 2.0 / 3.0) < 1e-15
    rng = np.random.default_rng(0)
    rec[:, 2] = np.round(rng.normal(0, 400, size=1000)).astype(np.int64)
    big = O.Params(L=64, T=1.0)
    rec2 = np.zeros((200000, 5), dtype=np.int64)
    rec2[:, 2] = np.round(rng.normal(0, 400, size=200000)).astype(np.int64)
    assert abs(OB.statistics(big, rec2)["binder"]) < 0.02


@pytest.mark.parametrize("T,sweeps,burn", [(2.6, 40000, 2000), (2.0, 40000, 2000)])
def test_oracle_run_matches_kaufman(T, sweeps, burn):
    """64 x 64 spin-1/2 at T away from T_c: mean energy and heat capacity
    equal Kaufman's finite-size values within 4 blocked standard errors."""
    p = O.Params(L=64, T=T, seed=123, init=O.INIT_COLD)
    s = O.init_lattice(p)
    rec = O.run(p, s, 0, sweeps)[burn:]
    N = 64 * 64
    e = -rec[:, 1] / N
    e_exact, c_exact = kaufman_energy_heat(64, T)
    mean, err = blocked_mean_err(e)
    assert abs(mean - e_exact) < 4 * err + 1e-6, (mean, e_exact, err)
    st = OB.statistics(p, rec)
    # heat capacity: error from the blocked error of (e - <e>)^2
    dev2 = N * (e - mean) ** 2 / (T * T)
    c_mean, c_err = blocked_mean_err(dev2)
    assert abs(st["heat_capacity"] - c_mean) < 1e-9 * c_mean
    assert abs(c_mean - c_exact) < 4 * c_err, (c_mean, c_exact, c_err)


def test_autocorrelation_limits():
    p = O.Params(model=O.NORTH_EAST, L=64, c=0.2, seed=3)
    s = O.init_lattice(p)
    assert OB.autocorrelation(p, OB.overlap(p, s, s)) == pytest.approx(1.0, abs=1e-15)
    # independent Bernoulli(c) states: Phi ~ 0 within a few / sqrt(N)
    vals = []
    for k in range(20):
        a = O.init_lattice(O.Params(model=O.NORTH_EAST, L=64, c=0.2, seed=100 + 2 * k))
        b = O.init_lattice(O.Params(model=O.NORTH_EAST, L=64, c=0.2, seed=101 + 2 * k))
        vals.append(OB.autocorrelation(p, OB.overlap(p, a, b)))
    assert abs(np.mean(vals)) < 4.0 / math.sqrt(64 * 64 * len(vals))
    # Ising overlap of a state with itself counts every spin-1/2 site once
    pi = O.Params(L=16, seed=1)
    si = O.init_lattice(pi)
    assert OB.overlap(pi, si, si) == 256
    assert OB.overlap(pi, si, -si) == -256


def test_spin_values_of_ne_bytes_ignore_the_flag():
    p = O.Params(model=O.NORTH_EAST, L=8, c=0.3)
    s = np.array([[0, 1, 2, 3] * 2] * 8, dtype=np.int8)
    v = OB.spin_values(p, s)
    assert v.tolist()[0] == [-1, 1, -1, 1] * 2


def test_oracle_run_matches_kaufman_at_the_c1_temperature():
    """64 x 64 from a cold start at T = 2.269 (the small parity configuration's
    lattice and temperature, next to T_c): mean energy per site equals Kaufman's
    finite-size value within 4 blocked standard errors."""
    p = O.Params(L=64, T=2.269, seed=1, init=O.INIT_COLD)
    s = O.init_lattice(p)
    rec = O.run(p, s, 0, 150000)[10000:]
    e = -rec[:, 1] / 4096.0
    e_exact, _ = kaufman_energy_heat(64, 2.269)
    mean, err = blocked_mean_err(e, nblocks=28)
    assert err < 2e-3
    assert abs(mean - e_exact) < 4 * err, (mean, e_exact, err)
