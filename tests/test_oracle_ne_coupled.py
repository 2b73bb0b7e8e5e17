"""Pins of the oracle's North-East model with the Ising coupling (Sec. 3.2, J != 0).

The coupled model moves an NE site only when its north and east neighbours
are up, and then with the Metropolis probability of the Ising energy
E = -J sum s_i s_j - h sum s_i over s = 2n - 1 (the thermodynamics of the
Ising model under the NE constraint).  The expected values come from:
  - the J = 0 NE model (pinned in test_oracle_pins.py), which the coupled
    model must reproduce bit for bit at J = 0, h = -1 and the T of c;
  - the deterministic limits T -> infinity (every allowed move) and T -> 0
    (an allowed move iff it does not raise the energy), with energies
    computed by brute force over all bonds;
  - exact enumeration of the 4x4 Boltzmann weights: each move is reversible,
    and a long run averages them over the states the constraint lets it reach.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle as O
import oracle.observables as OB
from exact import blocked_mean_err


def _colours(shape):
    return np.indices(shape).sum(axis=0) & 1


def _spins(b):
    return 2 * (b.astype(np.int64) & 1) - 1


def _energy(s, J, h):
    """E = -J sum over forward bonds s_i s_j - h sum s_i, by brute force."""
    bonds = np.sum(s * np.roll(s, -1, axis=0)) + np.sum(s * np.roll(s, -1, axis=1))
    return -J * float(bonds) - h * float(np.sum(s))


def _allowed(n):
    """North (y-1) and east (x+1) neighbours both up."""
    return (np.roll(n, 1, axis=0) & np.roll(n, -1, axis=1)).astype(bool)


def _coupled(**kw):
    base = dict(model=O.NE_COUPLED, L=16, J=1.0, h=0.0, T=3.0, c=0.5, seed=1)
    base.update(kw)
    return O.Params(**base)


def test_zero_coupling_reproduces_the_ne_model():
    """J = 0, h = -1 (one unit of energy per up site) at T = 2 / ln((1-c)/c):
    the up-flip probability e^{-2/T} equals c/(1-c) and down-flips are always
    accepted, so the run equals the J = 0 NE run from the same seed (the two
    thresholds may differ by one unit of 2^-32 from rounding, which no word of
    this short run hits)."""
    for c in (0.1, 0.3):
        T = 2.0 / math.log((1.0 - c) / c)
        q = _coupled(L=32, J=0.0, h=-1.0, T=T, c=c, seed=5)
        p = O.Params(model=O.NORTH_EAST, L=32, c=c, seed=5)
        tab = O.threshold_table(q).astype(np.int64)
        ne = O.threshold_table(p).astype(np.int64)
        z = 4
        for nsum in range(-z, z + 1):
            assert abs(tab[3 * (2 * z + 1) + nsum + z] - ne[0]) <= 1  # up-flip, ds = +2
            assert tab[0 * (2 * z + 1) + nsum + z] == ne[1] == 2 ** 32  # down-flip
        a, b = O.init_lattice(q), O.init_lattice(p)
        np.testing.assert_array_equal(a, b)
        ra = O.run(q, a, 0, 30)
        rb = O.run(p, b, 0, 30)
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(ra, rb)


def test_infinite_temperature_is_the_constrained_automaton():
    """T -> infinity: every allowed site changes, n <- n xor (north and east)."""
    q = _coupled(L=12, J=1.0, h=0.4, T=1e300, c=0.6, seed=2)
    s = O.init_lattice(q)
    ref = s.copy()
    col = _colours(ref.shape)
    O.run(q, s, 0, 6, records=False)
    for _ in range(6):
        for c in (0, 1):
            flip = _allowed(ref & 1) & (col == c)
            ref[flip] = ((ref[flip] & 1) ^ 1) | 2
    np.testing.assert_array_equal(s, ref)


@pytest.mark.parametrize("J,h", [(1.0, 0.0), (1.0, 0.3), (-0.7, 0.2), (0.5, -1.1)])
def test_zero_temperature_is_the_greedy_constrained_automaton(J, h):
    """T -> 0+: an allowed site changes iff that does not raise the energy; the
    energy change is the brute-force difference of the whole lattice's E."""
    q = _coupled(L=8, J=J, h=h, T=1e-300, c=0.55, seed=3)
    s = O.init_lattice(q)
    ref = s.copy()
    col = _colours(ref.shape)
    O.run(q, s, 0, 4, records=False)
    for _ in range(4):
        for c in (0, 1):
            allowed = _allowed(ref & 1) & (col == c)
            new = ref.copy()
            for y, x in zip(*np.nonzero(allowed)):
                before = _spins(ref)
                after = before.copy()
                after[y, x] = -after[y, x]
                if _energy(after, J, h) - _energy(before, J, h) <= 0.0:
                    new[y, x] = ((ref[y, x] & 1) ^ 1) | 2
            ref = new
    np.testing.assert_array_equal(s, ref)


def test_moves_are_reversible_for_the_boltzmann_weights_4x4():
    """Each allowed move of the coupled model satisfies detailed balance with
    respect to exp(-E/T) (E by brute force on every 4x4 state); the
    constraint does not involve the moving site, so it is symmetric."""
    for J, h, T in ((1.0, 0.0, 2.269), (1.0, 0.25, 1.7), (-0.6, -0.3, 2.5)):
        q = _coupled(L=4, J=J, h=h, T=T)
        tab = O.threshold_table(q) / 2 ** 32
        n = 16
        idx = np.arange(2 ** n)
        occ = ((idx[:, None] >> np.arange(n)) & 1).reshape(-1, 4, 4)
        s = 2 * occ - 1
        E = -J * (np.sum(s * np.roll(s, -1, axis=1), axis=(1, 2)) +
                  np.sum(s * np.roll(s, -1, axis=2), axis=(1, 2))) - h * np.sum(s, axis=(1, 2))
        logw = -E / T
        pi = np.exp(logw - logw.max())
        pi /= pi.sum()
        allowed = (np.roll(occ, 1, axis=1) & np.roll(occ, -1, axis=2)).reshape(-1, n)
        nsum = sum(np.roll(s, d, axis=ax) for ax in (1, 2) for d in (1, -1)).reshape(-1, n)
        flat = s.reshape(-1, n)
        z = 4
        di = np.where(flat > 0, 0, 3)  # ds = -2 for s = +1, +2 for s = -1
        acc = np.where(allowed == 1, tab[di * (2 * z + 1) + nsum + z], 0.0)
        for i in range(n):
            j = idx ^ (1 << i)
            lhs, rhs = pi * acc[:, i], pi[j] * acc[j, i]
            assert np.max(np.abs(lhs - rhs) / np.maximum(np.maximum(lhs, rhs), 1e-300)) < 1e-8


def test_flip_frequencies_follow_the_metropolis_rule():
    """One fixed state, many sweep indices: each site of colour 0 changes with
    probability [north and east up] min(1, exp(-dE/T)), dE by brute force."""
    J, h, T = 1.0, 0.2, 2.0
    q = _coupled(L=8, J=J, h=h, T=T, c=0.6, seed=9)
    s0 = O.init_lattice(q)
    col = _colours(s0.shape)
    trials = 4000
    flips = np.zeros(s0.shape)
    for t in range(trials):
        s = s0.copy()
        O.half_sweep(q, s, t, 0)
        flips += (s & 1) != (s0 & 1)
    allowed = _allowed(s0 & 1)
    sp = _spins(s0)
    e0 = _energy(sp, J, h)
    for y, x in zip(*np.nonzero(col == 0)):
        if not allowed[y, x]:
            assert flips[y, x] == 0
            continue
        after = sp.copy()
        after[y, x] = -after[y, x]
        pr = min(1.0, math.exp(-(_energy(after, J, h) - e0) / T))
        sd = math.sqrt(max(pr * (1 - pr), 1e-12) / trials)
        assert abs(flips[y, x] / trials - pr) < 4.5 * sd + 1e-9, (y, x, flips[y, x] / trials, pr)


def test_spin_sums_of_ne_records():
    """Records count over n; spin_sums turns them into sums over s = 2n - 1."""
    q = _coupled(L=12, c=0.35, seed=4)
    s = O.init_lattice(q)
    O.run(q, s, 0, 3, records=False)
    rec = O.initial_record(q, s)[None, :]
    bond, mag = OB.spin_sums(q, rec)
    sp = _spins(s)
    assert bond[0] == np.sum(sp * np.roll(sp, -1, 0)) + np.sum(sp * np.roll(sp, -1, 1))
    assert mag[0] == np.sum(sp)


def _frozen_down(occ):
    """Down sites that can never move: the largest set of down sites each of
    whose north or east neighbour is in the set (a directed down cycle that
    wraps the torus, with what hangs on it).  Such a set can be neither
    created nor removed by the constrained dynamics, so the states without
    one form the component of the all-up state."""
    f = (occ == 0)
    while True:
        g = f & (np.roll(f, 1, axis=-2) | np.roll(f, -1, axis=-1))
        if np.array_equal(g, f):
            return f
        f = g


@pytest.mark.parametrize("J,h,T", [(1.0, 0.0, 2.5), (1.0, 0.3, 2.0), (-0.5, 0.2, 1.5)])
def test_equilibrium_4x4_matches_enumeration_of_its_component(J, h, T):
    """The constrained dynamics keeps exp(-E/T) restricted to the states it
    can reach.  From the all-up state those are the 4x4 states with no frozen
    down set; exact averages over them (brute-force E) against a long run."""
    n = 16
    idx = np.arange(2 ** n)
    occ = ((idx[:, None] >> np.arange(n)) & 1).reshape(-1, 4, 4)
    free = ~_frozen_down(occ).reshape(-1, n).any(axis=1)
    s = 2 * occ - 1
    bond = (np.sum(s * np.roll(s, -1, axis=1), axis=(1, 2)) +
            np.sum(s * np.roll(s, -1, axis=2), axis=(1, 2)))
    mag = np.sum(s, axis=(1, 2))
    E = -J * bond - h * mag
    logw = np.where(free, -E / T, -np.inf)
    w = np.exp(logw - logw[free].max())
    w /= w.sum()
    e_ex, m_ex = float(np.sum(w * E)) / n, float(np.sum(w * mag)) / n
    q = _coupled(L=4, J=J, h=h, T=T, c=0.999, seed=17)
    lat = O.init_lattice(q)
    assert not _frozen_down(lat & 1).any()
    rec = O.run(q, lat, 0, 200000)[1000:]
    b, m = OB.spin_sums(q, rec)
    e = (-J * b - h * m) / n
    for series, ex in ((e, e_ex), (m / n, m_ex)):
        mu, err = blocked_mean_err(series)
        assert abs(mu - ex) < 4 * err, (mu, ex, err)
    assert abs(OB.statistics(q, rec)["e"] - float(np.mean(e))) < 1e-12


def test_thread_count_and_split_runs():
    """The coupled half-sweep reads only the other colour, so the OpenMP thread
    count and where a run is split cannot change the result."""
    q = _coupled(L=32, J=1.0, h=0.1, T=2.2, c=0.6, seed=12)
    a = O.init_lattice(q)
    b, c = a.copy(), a.copy()
    ra = O.run(q, a, 0, 20, nthreads=1)
    rb = O.run(q, b, 0, 20, nthreads=4)
    rc = np.vstack([O.run(q, c, 0, 7, nthreads=2), O.run(q, c, 7, 13, nthreads=3)])
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a, c)
    np.testing.assert_array_equal(ra, rb)
    np.testing.assert_array_equal(ra, rc)
