"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test names what fixes the expected value: rocRAND's independent
Philox4x32-10, high-precision evaluation of the Metropolis rule, limits in
which the sweep is a deterministic cellular automaton, exact enumeration of
small lattices, Onsager's and Yang's closed forms, the balance property of
the checkerboard kernel (paper Sec. 3.1: the GPU order keeps balance but not
detailed balance), and the kinetic constraint of the North-East model.
"""
from __future__ import annotations

import math
import os
import subprocess
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle as O
import exact as X

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# ---------------------------------------------------------------------------
# Philox4x32-10 against rocRAND's implementation (called, not copied)

@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_philox_ref")
    src = os.path.join(ROOT, "tests", "rocrand_philox_ref.cpp")
    subprocess.check_call(["/opt/rocm/bin/hipcc", "-O1", "-x", "hip", "--offload-arch=gfx950",
                           src, "-o", exe], stderr=subprocess.DEVNULL)
    return exe


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(1234)
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF,) * 6, (1, 0, 0, 0, 0, 0), (0, 0, 0, 1, 0, 0),
             (0, 0, 0, 0, 0, 1), (5, 1, 2269, 0, 1, 0), (123, 0, 99, 1, 1, 0)]
    cases += [tuple(int(v) for v in row) for row in rng.integers(0, 2 ** 32, size=(600, 6))]
    inp = "".join(" ".join(str(v) for v in c) + "\n" for c in cases)
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [list(map(int, line.split())) for line in out.strip().splitlines()]
    assert len(ref) == len(cases)
    for c, r in zip(cases, ref):
        assert O.philox4x32_10(c[:4], c[4:]) == r, c


def test_rand_word_selects_contract_word():
    """word(seed, tag, t, colour, k, w, j) = Philox(ctr=(k//G, colour, t, tag))[(k%G)*w+j]."""
    seed = (7 << 32) | 3
    for w in (1, 2):
        G = 4 // w
        for k in (0, 1, 2, 3, 4, 5, 1001, 2 ** 20 + 3):
            for j in range(w):
                block = O.philox4x32_10((k // G, 1, 42, 0), (3, 7))
                assert O.rand_word(seed, 0, 42, 1, k, w, j) == block[(k % G) * w + j]


# ---------------------------------------------------------------------------
# Metropolis thresholds: floor(min(1, e^{-dE/T}) 2^32) against 50-digit exp

def _thr_exact(dE, T):
    getcontext().prec = 60
    if dE <= 0:
        return 2 ** 32
    p = (Decimal(-dE) / Decimal(T)).exp()
    return int((p * (2 ** 32)).to_integral_value(rounding="ROUND_FLOOR"))


@pytest.mark.parametrize("T", [2.0, 2.269, 2.6, 0.7, 4.5115])
def test_threshold_matches_high_precision(T):
    for dE in (0.5, 1.0, 2.0, 4.0, 6.0, 8.0, 12.0):
        assert O.threshold(dE, T) == _thr_exact(dE, Decimal(repr(T))), (dE, T)
    assert O.threshold(0.0, T) == 2 ** 32
    assert O.threshold(-4.0, T) == 2 ** 32


def test_threshold_table_layout_2d_spin_half():
    """Flipping s=+1 with all four neighbours +1 costs dE = 2*J*4 = 8 (Eq. 2):
    entry [ds=-2][nsum=+4]; flipping it against four -1 neighbours gains 8."""
    for T in (2.0, 2.269, 2.6):
        tab = O.threshold_table(O.Params(T=T))
        z = 4
        col = 2 * z + 1
        assert len(tab) == 4 * col
        assert tab[0 * col + (4 + z)] == _thr_exact(8, Decimal(repr(T)))
        assert tab[0 * col + (2 + z)] == _thr_exact(4, Decimal(repr(T)))
        assert tab[0 * col + (-4 + z)] == 2 ** 32
        # s=-1 -> +1 (ds=+2) against four -1 neighbours (nsum=-4) costs 8
        assert tab[3 * col + (-4 + z)] == _thr_exact(8, Decimal(repr(T)))


def test_threshold_field_sign():
    """H = -J sum s s - h sum s: with h > 0 and no neighbours' preference,
    turning +1 into -1 costs 2h."""
    tab = O.threshold_table(O.Params(T=1.0, J=1.0, h=0.25))
    z, col = 4, 9
    assert tab[0 * col + (0 + z)] == _thr_exact(0.5, Decimal(1))
    assert tab[3 * col + (0 + z)] == 2 ** 32


def test_ne_thresholds():
    """NE: up-flips with probability c/(1-c), down-flips always for c < 1/2."""
    for c in (0.05, 0.1, 0.2):
        tab = O.threshold_table(O.Params(model=O.NORTH_EAST, c=c))
        getcontext().prec = 60
        cd = Decimal(repr(c))
        # c/(1-c) evaluated as the double quotient, floor(2^32 * it) exactly
        ratio = c / (1.0 - c)
        assert tab[0] == int((Decimal(ratio) * 2 ** 32).to_integral_value(rounding="ROUND_FLOOR"))
        assert abs(int(tab[0]) / 2 ** 32 - float(cd / (1 - cd))) < 1e-9
        assert tab[1] == 2 ** 32
    assert O.threshold_table(O.Params(model=O.NORTH_EAST, c=0.2))[0] == 2 ** 30


# ---------------------------------------------------------------------------
# Deterministic limits: the sweep becomes a cellular automaton

def _np_colours(shape):
    grids = np.indices(shape)
    return grids.sum(axis=0) & 1


def _np_nsum(s):
    tot = np.zeros(s.shape, dtype=np.int64)
    for ax in range(s.ndim):
        tot += np.roll(s, 1, axis=ax) + np.roll(s, -1, axis=ax)
    return tot


def _zero_T_sweep(s, J, h):
    """T -> 0+: accept iff dE <= 0 with dE = 2 s (J nsum + h); colour 0 first."""
    col = _np_colours(s.shape)
    s = s.astype(np.int64).copy()
    for c in (0, 1):
        dE = 2.0 * s * (J * _np_nsum(s) + h)
        flip = (col == c) & (dE <= 0)
        s[flip] = -s[flip]
    return s.astype(np.int8)


@pytest.mark.parametrize("dim,L,h", [(2, 8, 0.0), (2, 10, 0.3), (3, 6, 0.0), (3, 4, -0.2)])
def test_zero_temperature_is_greedy_automaton(dim, L, h):
    p = O.Params(dim=dim, L=L, T=1e-6, h=h, seed=5)
    s = O.init_lattice(p)
    ref = s.copy()
    O.run(p, s, 0, 6, records=False)
    for _ in range(6):
        ref = _zero_T_sweep(ref, 1.0, h)
    np.testing.assert_array_equal(s, ref)


@pytest.mark.parametrize("dim,L", [(2, 8), (2, 6), (3, 4)])
def test_infinite_temperature_flips_every_spin(dim, L):
    p = O.Params(dim=dim, L=L, T=math.inf, seed=9)
    s = O.init_lattice(p)
    s0 = s.copy()
    rec = O.run(p, s, 0, 1)
    np.testing.assert_array_equal(s, -s0)
    assert rec[0, 3] == p.nsites


def test_infinite_temperature_spin_one_always_moves():
    p = O.Params(L=8, two_s=2, T=math.inf, seed=4)
    s = O.init_lattice(p)
    s0 = s.copy()
    rec = O.run(p, s, 0, 1)
    assert np.all(s != s0) and rec[0, 3] == p.nsites
    assert set(np.unique(s)).issubset({-1, 0, 1})


def test_cold_start_is_fixed_at_low_temperature():
    p = O.Params(L=16, T=1e-6, init=O.INIT_COLD)
    s = O.init_lattice(p)
    assert np.all(s == 1)
    rec = O.run(p, s, 0, 3)
    assert np.all(s == 1)
    assert np.all(rec[:, 1] == 2 * p.nsites) and np.all(rec[:, 2] == p.nsites)
    assert np.all(rec[:, 3] == 0)


def _ne_ca_sweep(b):
    """c = 1/2: every allowed move is accepted, so a half-sweep is the automaton
    n <- n xor (n_north and n_east) on one colour (north = y-1, east = x+1)."""
    col = _np_colours(b.shape)
    b = b.copy()
    for c in (0, 1):
        n = b & 1
        allowed = (np.roll(n, 1, axis=0) & np.roll(n, -1, axis=1)).astype(bool) & (col == c)
        b[allowed] = ((b[allowed] & 1) ^ 1) | 2
    return b


def test_ne_half_density_is_automaton():
    p = O.Params(model=O.NORTH_EAST, L=12, c=0.5, seed=2)
    s = O.init_lattice(p)
    ref = s.copy()
    O.run(p, s, 0, 5, records=False)
    for _ in range(5):
        ref = _ne_ca_sweep(ref)
    np.testing.assert_array_equal(s, ref)


def test_ne_constraint_blocks_moves():
    """A site whose north or east neighbour is down never changes."""
    p = O.Params(model=O.NORTH_EAST, L=16, c=0.3, seed=8)
    s = O.init_lattice(p)
    col = _np_colours(s.shape)
    for t in range(10):
        for c in (0, 1):
            before = s.copy()
            O.half_sweep(p, s, t, c)
            n = before & 1
            blocked = ~(np.roll(n, 1, axis=0) & np.roll(n, -1, axis=1)).astype(bool)
            assert np.all(s[blocked | (col != c)] == before[blocked | (col != c)])


# ---------------------------------------------------------------------------
# Records: brute-force recount against numpy definitions

@pytest.mark.parametrize("model,dim,two_s", [(0, 2, 1), (0, 2, 2), (0, 3, 1), (1, 2, 1)])
def test_recount_matches_definition(model, dim, two_s):
    p = O.Params(model=model, dim=dim, L=6, two_s=two_s, c=0.4, T=3.0, seed=3)
    s = O.init_lattice(p)
    O.run(p, s, 0, 3, records=False)
    b, m, u = O.recount(p, s)
    v = (s & 1) if model == 1 else s.astype(np.int64)
    v = v.astype(np.int64)
    bond = sum(int(np.sum(v * np.roll(v, -1, axis=ax))) for ax in range(dim))
    assert b == bond and m == int(v.sum())
    if model == 1:
        assert u == int(np.sum((s & 2) == 0))
    else:
        assert u == -1


def test_ne_persistence_monotone_and_reset():
    p = O.Params(model=O.NORTH_EAST, L=32, c=0.2, seed=1)
    s = O.init_lattice(p)
    assert O.recount(p, s)[2] == p.nsites  # P(t0) = 1
    rec = O.run(p, s, 0, 50)
    assert np.all(np.diff(rec[:, 4]) <= 0)
    O.reset_persistence(p, s)
    assert O.recount(p, s)[2] == p.nsites


# ---------------------------------------------------------------------------
# Schedule independence of the oracle itself

def test_thread_count_and_split_runs():
    p = O.Params(L=32, T=2.269, seed=12)
    a = O.init_lattice(p)
    b = a.copy()
    c = a.copy()
    ra = O.run(p, a, 0, 20, nthreads=1)
    rb = O.run(p, b, 0, 20, nthreads=4)
    rc = np.vstack([O.run(p, c, 0, 7, nthreads=2), O.run(p, c, 7, 13, nthreads=3)])
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a, c)
    np.testing.assert_array_equal(ra, rb)
    np.testing.assert_array_equal(ra, rc)


# ---------------------------------------------------------------------------
# Transition probabilities of one half-sweep, measured over many seeds

def test_half_sweep_flip_frequencies():
    """Each colour-0 site flips with probability thr(dE)/2^32 (binomial, 4 sigma)."""
    p = O.Params(L=8, T=2.0, seed=0)
    start = O.init_lattice(O.Params(L=8, seed=77))
    col = _np_colours(start.shape)
    nsum = _np_nsum(start.astype(np.int64))
    dE = 2.0 * start * nsum
    prob = np.array([O.threshold(float(e), 2.0) for e in dE.ravel()]).reshape(dE.shape) / 2 ** 32
    trials = 3000
    flips = np.zeros(start.shape)
    for seed in range(trials):
        q = O.Params(L=8, T=2.0, seed=seed + 1000)
        s = start.copy()
        O.half_sweep(q, s, 0, 0)
        flips += (s != start)
    assert np.all(flips[col == 1] == 0)
    pm = prob[col == 0]
    sigma = np.sqrt(trials * pm * (1 - pm)) + 1e-9
    assert np.all(np.abs(flips[col == 0] - trials * pm) <= 4 * sigma + 1e-9)


def test_half_sweep_spin_one_proposals():
    """Spin-1 at T = inf: each proposal value is taken with probability 1/2."""
    start = np.zeros((8, 8), dtype=np.int8)
    col = _np_colours(start.shape)
    trials = 2000
    ups = np.zeros(start.shape)
    for seed in range(trials):
        q = O.Params(L=8, two_s=2, T=math.inf, seed=seed + 1)
        s = start.copy()
        O.half_sweep(q, s, 0, 0)
        assert np.all(s[col == 0] != 0)
        ups += (s == 1)
    frac = ups[col == 0] / trials
    assert np.all(np.abs(frac - 0.5) < 4 * math.sqrt(0.25 / trials))


# ---------------------------------------------------------------------------
# Balance of the checkerboard kernel (paper Sec. 3.1): exact, on 4x4 spin-1/2

def test_checkerboard_kernel_balance_4x4():
    T = 2.269
    shape = (4, 4)
    n = 16
    idx = np.arange(2 ** n)
    spins = (1 - 2 * ((idx[:, None] >> np.arange(n)) & 1)).reshape(-1, 4, 4)
    bond = sum(np.sum(spins * np.roll(spins, -1, axis=ax), axis=(1, 2)) for ax in (1, 2))
    logw = bond / T
    pi = np.exp(logw - logw.max())
    pi /= pi.sum()
    col = _np_colours(shape).ravel()
    nsum = np.zeros((2 ** n, n))
    for ax in (1, 2):
        nsum += (np.roll(spins, 1, axis=ax) + np.roll(spins, -1, axis=ax)).reshape(-1, n)
    flat = spins.reshape(-1, n)
    dE = 2.0 * flat * nsum
    table = {e: O.threshold(float(e), T) / 2 ** 32 for e in np.unique(dE)}
    acc = np.vectorize(table.get)(dE)  # acceptance of flipping site i from state x
    # each single-site move is reversible w.r.t. pi (Metropolis, up to 2^-32)
    for i in range(n):
        j = idx ^ (1 << i)
        lhs = pi * acc[:, i]
        rhs = pi[j] * acc[j, i]
        assert np.max(np.abs(lhs - rhs) / np.maximum(lhs, 1e-300)) < 1e-8
    # a sweep applies colour 0 then colour 1 site moves: pi stays invariant
    v = pi.copy()
    for c in (0, 1):
        for i in np.nonzero(col == c)[0]:
            j = idx ^ (1 << i)
            v = v * (1 - acc[:, i]) + v[j] * acc[j, i]
    # each threshold is below e^{-dE/T} 2^32 by less than 1, so each of the 16
    # moves perturbs the invariant vector by less than 2^-32 of the mass moved
    assert np.max(np.abs(v - pi)) < 16 * 2.0 ** -32
    # ... but the full sweep is not reversible: K(x,y) = K0(x,z) K1(z,y) with
    # z = (colour-0 part of y, colour-1 part of x)
    def kernel(x, y):
        z = (y & m0) | (x & m1)
        k = 1.0
        for i in range(n):
            a_xz = acc[x, i] if col[i] == 0 else acc[z, i]
            flip = ((x if col[i] == 0 else z) ^ (z if col[i] == 0 else y)) >> i & 1
            k *= a_xz if flip else (1 - a_xz)
        return k
    m0 = int(sum(1 << i for i in range(n) if col[i] == 0))
    m1 = (2 ** n - 1) ^ m0
    rng = np.random.default_rng(0)
    worst = 0.0
    for _ in range(200):
        x, y = (int(v) for v in rng.integers(0, 2 ** n, size=2))
        f, b = pi[x] * kernel(x, y), pi[y] * kernel(y, x)
        if max(f, b) > 0:
            worst = max(worst, abs(f - b) / max(f, b))
    assert worst > 0.1


# ---------------------------------------------------------------------------
# Equilibrium: oracle averages against exact enumeration (3 sigma, blocking)

def _mc(p, nsweeps, burn):
    s = O.init_lattice(p)
    rec = O.run(p, s, 0, nsweeps)[burn:]
    N = p.nsites
    return -rec[:, 1] / N, np.abs(rec[:, 2]) / N, (rec[:, 2] / N) ** 2


@pytest.mark.parametrize("T", [2.0, 2.269, 2.6])
def test_equilibrium_4x4_spin_half(T):
    b, m = X.enumerate_spin_half((4, 4))
    e_ex, am_ex, m2_ex, _ = X.canonical_averages(b, m, T, 16)
    e, am, m2 = _mc(O.Params(L=4, T=T, seed=21), 200000, 1000)
    for series, ex in ((e, e_ex), (am, am_ex), (m2, m2_ex)):
        mu, err = X.blocked_mean_err(series)
        assert abs(mu - ex) < 3 * err, (mu, ex, err)


def test_equilibrium_4x4_spin_one():
    T = 1.6935
    b, m, g = X.enumerate_spin_one_4x4()
    e_ex, am_ex, _, _ = X.canonical_averages(b, m, T, 16, weight=g)
    e, am, _ = _mc(O.Params(L=4, two_s=2, T=T, seed=22), 200000, 1000)
    for series, ex in ((e, e_ex), (am, am_ex)):
        mu, err = X.blocked_mean_err(series)
        assert abs(mu - ex) < 3 * err, (mu, ex, err)


def test_equilibrium_2x2x2_spin_half():
    T = 4.5115
    b, m = X.enumerate_spin_half((2, 2, 2))
    e_ex, am_ex, _, _ = X.canonical_averages(b, m, T, 8)
    e, am, _ = _mc(O.Params(dim=3, L=2, T=T, seed=23), 200000, 1000)
    for series, ex in ((e, e_ex), (am, am_ex)):
        mu, err = X.blocked_mean_err(series)
        assert abs(mu - ex) < 3 * err, (mu, ex, err)


# ---------------------------------------------------------------------------
# Onsager / Yang on a 64x64 lattice (finite-size effects far below the error)

def test_onsager_energy_above_tc():
    e, _, _ = _mc(O.Params(L=64, T=2.6, seed=31), 4000, 500)
    mu, err = X.blocked_mean_err(e)
    assert abs(mu - X.onsager_energy(2.6)) < 3 * err, (mu, err)


def test_onsager_yang_below_tc_cold_start():
    p = O.Params(L=64, T=2.0, seed=32, init=O.INIT_COLD)
    e, am, _ = _mc(p, 4000, 500)
    mu, err = X.blocked_mean_err(e)
    assert abs(mu - X.onsager_energy(2.0)) < 3 * err, (mu, err)
    mu, err = X.blocked_mean_err(am)
    assert abs(mu - X.yang_magnetisation(2.0)) < 3 * err, (mu, err)


# ---------------------------------------------------------------------------
# North-East model: equilibrium density and the stuck fraction below c*

def test_ne_density_stationary():
    """Bernoulli(c) is invariant: starting from one equilibrium sample the mean
    density stays c within the spread of such a sample, sqrt(c(1-c)/N) (below
    c* the dynamics barely moves the density, so time averages do not shrink
    that spread)."""
    c = 0.2
    p = O.Params(model=O.NORTH_EAST, L=256, c=c, seed=41)
    s = O.init_lattice(p)
    rec = O.run(p, s, 0, 200)
    dens = rec[:, 2] / p.nsites
    assert abs(dens.mean() - c) < 3 * math.sqrt(c * (1 - c) / p.nsites)


def test_ne_moves_balance_product_measure():
    """Each NE move is reversible w.r.t. prod_i c^n_i (1-c)^(1-n_i) (the
    constraint does not involve the site): exact check on all 4x4 states."""
    for c in (0.1, 0.3, 0.6):
        tab = O.threshold_table(O.Params(model=O.NORTH_EAST, c=c)) / 2 ** 32
        n = 16
        idx = np.arange(2 ** n)
        occ = ((idx[:, None] >> np.arange(n)) & 1).reshape(-1, 4, 4)
        k = occ.reshape(-1, n).sum(axis=1)
        pi = c ** k * (1 - c) ** (n - k)
        allowed = (np.roll(occ, 1, axis=1) & np.roll(occ, -1, axis=2)).reshape(-1, n)
        flat = occ.reshape(-1, n)
        for i in range(n):
            a = np.where(allowed[:, i] == 1, np.where(flat[:, i] == 1, tab[1], tab[0]), 0.0)
            j = idx ^ (1 << i)
            assert np.max(np.abs(pi * a - pi[j] * a[j])) < 2.0 ** -31


def test_ne_persistence_plateau_below_critical_density():
    """c = 0.05 < c* ~ 0.3 (Sec. 5.2): a finite fraction of sites stays stuck."""
    p = O.Params(model=O.NORTH_EAST, L=64, c=0.05, seed=42)
    s = O.init_lattice(p)
    rec = O.run(p, s, 0, 3000)
    P = rec[:, 4] / p.nsites
    assert P[-1] > 0.5 and abs(P[-1] - P[-1000]) < 0.02


# ---------------------------------------------------------------------------
# Conventions of the random-number contract that physics cannot see: the
# initial-state rule, the spin-1 proposal rule and the strict comparison.
# Words come from rand_word, itself pinned to rocRAND above.

def _colour_index(shape):
    col = _np_colours(shape)
    k = np.arange(int(np.prod(shape))).reshape(shape) >> 1
    return col, k


@pytest.mark.parametrize("model,dim,two_s", [(0, 2, 1), (0, 2, 2), (0, 3, 1), (0, 3, 2), (1, 2, 1)])
def test_initial_state_contract(model, dim, two_s):
    p = O.Params(model=model, dim=dim, L=6, two_s=two_s, c=0.3, seed=(5 << 32) | 17)
    s = O.init_lattice(p)
    col, k = _colour_index(s.shape)
    bern = math.floor(0.3 * 2 ** 32)
    for i in np.ndindex(s.shape):
        u = O.rand_word(p.seed, 1, 0, int(col[i]), int(k[i]), 1, 0)
        if model == 1:
            want = 1 if u < bern else 0
        elif two_s == 1:
            want = 1 if u < 2 ** 31 else -1
        else:
            want = (u * 3 >> 32) - 1
        assert s[i] == want, i


def test_spin_one_proposal_contract():
    """T = inf accepts everything, so the new value is the proposal: the lower
    of the two other values iff word j=1 < 2^31."""
    p = O.Params(L=6, two_s=2, T=math.inf, seed=99)
    s = O.init_lattice(p)
    start = s.copy()
    O.half_sweep(p, s, 3, 1)
    col, k = _colour_index(s.shape)
    for i in np.ndindex(s.shape):
        if col[i] != 1:
            continue
        others = sorted({-1, 0, 1} - {int(start[i])})
        up = O.rand_word(p.seed, 0, 3, 1, int(k[i]), 2, 1)
        assert s[i] == (others[0] if up < 2 ** 31 else others[1])


def _temperature_with_threshold(dE, target):
    """Bisect T so that floor(exp(-dE/T) 2^32) == target (thresholds rise with T)."""
    lo, hi = 1e-3, 1e3
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if O.threshold(dE, mid) < target:
            lo = mid
        else:
            hi = mid
    for T in (lo, hi):
        if O.threshold(dE, T) == target:
            return T
    raise AssertionError("no temperature hits the target threshold")


def test_acceptance_is_strict_at_the_threshold():
    """A move whose word equals its threshold is rejected; one below is taken."""
    seed, t = 3, 0
    k = 5  # colour-0 site with in-colour index 5 of a cold 8x8 lattice
    u = O.rand_word(seed, 0, t, 0, k, 1, 0)
    col, kk = _colour_index((8, 8))
    site = tuple(int(v) for v in np.argwhere((col == 0) & (kk == k))[0])
    for target, flips in ((u, False), (u + 1, True)):
        T = _temperature_with_threshold(8.0, target)
        p = O.Params(L=8, T=T, seed=seed, init=O.INIT_COLD)
        s = O.init_lattice(p)
        O.half_sweep(p, s, t, 0)
        assert (s[site] == -1) == flips
    # NE: choose c so that floor(c/(1-c) 2^32) == u for an up-flip
    p = O.Params(model=O.NORTH_EAST, L=8, c=0.3, seed=seed)
    start = np.ones((8, 8), dtype=np.int8)
    start[site] = 0
    for target, flips in ((u, False), (u + 1, True)):
        lo, hi = 1e-6, 0.5
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if O.threshold_from_prob(mid / (1 - mid)) < target:
                lo = mid
            else:
                hi = mid
        c = next(v for v in (lo, hi) if O.threshold_from_prob(v / (1 - v)) == target)
        q = O.Params(model=O.NORTH_EAST, L=8, c=c, seed=seed)
        s = start.copy()
        O.half_sweep(q, s, t, 0)
        assert ((s[site] & 1) == 1) == flips
