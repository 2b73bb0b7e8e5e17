"""Pins of the oracle's North-East sub-lattice algorithm (paper Sec. 3.2, the
NE algorithm with random sub-lattices and lambda concurrent threads).

What fixes the oracle here, independently of its own loop:
  * a launch with lambda = P/2 is one iteration in which every attempt reads
    the launch-start lattice, so its outcome is predicted site by site from the
    Philox words (Philox itself is pinned against rocRAND elsewhere);
  * the closed form for the fraction of distinct sites among P/2 uniform draws
    (sites drawn twice flip once);
  * the serial limit Q = lambda = 1, where the paper states the algorithm is
    serial and balanced: detailed balance with respect to the product measure
    Bernoulli(c), checked empirically on every pair of states of a 2x2 lattice;
  * locality: a sub-lattice sees nothing of the rest of the lattice but its
    north row and east column, as they were when the launch started;
  * parity and persistence-flag invariants of every launch.
"""
import math

import numpy as np
import pytest

import oracle as O

TAG_NE_TILES = 2


def _params(L, B, lam, c, seed=1):
    return O.Params(model=O.NE_TILES, dim=2, L=L, c=c, seed=seed, tile=B, lam=lam)


def _random_state(L, c, seed, flags=True):
    rng = np.random.default_rng(seed)
    n = (rng.random((L, L)) < c).astype(np.int8)
    if flags:
        n |= (rng.random((L, L)) < 0.5).astype(np.int8) << 1
    return np.ascontiguousarray(n)


def _words(p, tau, a, launch):
    w = O.philox4x32_10([tau, a // 2, launch, TAG_NE_TILES],
                        [p.seed & 0xFFFFFFFF, p.seed >> 32])
    return w[2 * (a % 2)], w[2 * (a % 2) + 1]


def _predict_one_iteration(p, src, launch):
    """lambda = P/2: one iteration; every attempt reads src."""
    L, B = p.L, p.tile
    P = B * B
    up_thr = O.threshold_from_prob(p.c / (1 - p.c))
    down_thr = O.threshold_from_prob((1 - p.c) / p.c)
    n = src & 1
    north = np.roll(n, 1, axis=0)   # north of (x, y) is (x, y-1)
    east = np.roll(n, -1, axis=1)   # east of (x, y) is (x+1, y)
    flip = np.zeros((L, L), dtype=bool)
    for tau in range((L // B) ** 2):
        x0, y0 = (tau % (L // B)) * B, (tau // (L // B)) * B
        for a in range(P // 2):
            ws, wa = _words(p, tau, a, launch)
            site = (ws * P) >> 32
            y, x = y0 + site // B, x0 + site % B
            if not (north[y, x] and east[y, x]):
                continue
            thr = down_thr if n[y, x] else up_thr
            if wa < thr:
                flip[y, x] = True
    dst = src.copy()
    dst[flip] = ((src[flip] & 1) ^ 1) | 2
    return dst, int(flip.sum())


@pytest.mark.parametrize("L,B,c,launch", [(16, 8, 0.3, 7), (16, 4, 0.6, 0), (12, 4, 0.45, 123)])
def test_one_iteration_predicted_site_by_site(L, B, c, launch):
    p = _params(L, B, (B * B) // 2, c, seed=11)
    src = _random_state(L, 0.8, seed=L + B)
    dst, acc = O.ne_tiles_launch(p, src, launch)
    want, want_acc = _predict_one_iteration(p, src, launch)
    np.testing.assert_array_equal(dst, want)
    assert acc == want_acc


def test_sites_drawn_twice_flip_once():
    """c = 1/2 accepts every allowed move; on an all-up lattice every drawn
    site is allowed, so the changed fraction is the fraction of distinct sites
    among P/2 uniform draws: 1 - (1 - 1/P)^(P/2)."""
    L, B = 256, 8
    P = B * B
    p = _params(L, B, P // 2, 0.5, seed=5)
    src = np.ones((L, L), dtype=np.int8)
    dst, acc = O.ne_tiles_launch(p, src, 3)
    changed = int(((dst & 1) != 1).sum())
    assert acc == changed
    expect = 1 - (1 - 1 / P) ** (P // 2)
    sd = math.sqrt(expect * (1 - expect) / (L * L))  # draws of different tiles are independent
    assert abs(changed / (L * L) - expect) < 5 * sd + 1e-3
    # a toggle per draw (xor) would leave ~ (1 - e^{-1})/2 of the sites changed
    assert abs(changed / (L * L) - (1 - math.exp(-1)) / 2) > 0.05


def test_serial_limit_detailed_balance():
    """Q = lambda = 1 on a 2x2 lattice: the serial random-site algorithm, which
    the paper says preserves detailed balance.  pi(s) K(s,s') = pi(s') K(s',s)
    for the product measure pi = Bernoulli(c)^4, K estimated from many
    launches of every start state."""
    c, M = 0.3, 4000
    p = _params(2, 2, 1, c, seed=17)
    states = [np.array([[(v >> 0) & 1, (v >> 1) & 1], [(v >> 2) & 1, (v >> 3) & 1]],
                       dtype=np.int8) for v in range(16)]
    K = np.zeros((16, 16))
    for i, s in enumerate(states):
        for launch in range(M):
            d, _ = O.ne_tiles_launch(p, s, launch)
            d = d & 1
            j = int(d[0, 0]) | int(d[0, 1]) << 1 | int(d[1, 0]) << 2 | int(d[1, 1]) << 3
            K[i, j] += 1
    K /= M
    pi = np.array([c ** bin(v).count("1") * (1 - c) ** (4 - bin(v).count("1")) for v in range(16)])
    worst = 0.0
    for i in range(16):
        for j in range(16):
            if i == j:
                continue
            lhs, rhs = pi[i] * K[i, j], pi[j] * K[j, i]
            var = pi[i] ** 2 * K[i, j] * (1 - K[i, j]) / M + pi[j] ** 2 * K[j, i] * (1 - K[j, i]) / M
            if var == 0:
                assert lhs == rhs == 0
                continue
            worst = max(worst, abs(lhs - rhs) / math.sqrt(var))
    assert worst < 5.0
    # stationarity of pi under the launch
    assert np.abs(pi @ K - pi).max() < 0.01
    # the constraint forbids some moves: from the all-down state nothing changes
    assert K[0, 0] == 1.0


def test_sub_lattice_sees_only_its_north_row_and_east_column():
    L, B, lam = 24, 8, 4
    p = _params(L, B, lam, 0.35, seed=29)
    src = _random_state(L, 0.7, seed=3)
    dst, _ = O.ne_tiles_launch(p, src, 5)
    # tile tau = 4 is the centre one: rows 8..15, columns 8..15
    ys, xs = slice(8, 16), slice(8, 16)
    rng = np.random.default_rng(9)
    other = _random_state(L, 0.5, seed=4)
    keep = np.zeros((L, L), dtype=bool)
    keep[ys, xs] = True
    keep[7, 8:16] = True     # north row
    keep[8:16, 16] = True    # east column
    mixed = np.where(keep, src, other).astype(np.int8)
    d2, _ = O.ne_tiles_launch(p, np.ascontiguousarray(mixed), 5)
    np.testing.assert_array_equal(d2[ys, xs], dst[ys, xs])
    # with the north row and east column all down, the top row can only change
    # at columns whose east neighbour is inside the tile, and the east column
    # of the tile never changes
    blocked = src.copy()
    blocked[7, 8:16] = 0
    blocked[8:16, 16] = 0
    d3, _ = O.ne_tiles_launch(p, blocked, 5)
    assert np.array_equal(d3[8, 8:16], blocked[8, 8:16])
    assert np.array_equal(d3[8:16, 15], blocked[8:16, 15])
    del rng


@pytest.mark.parametrize("lam", [1, 2, 8, 32])
def test_launch_invariants(lam):
    L, B = 32, 8
    p = _params(L, B, lam, 0.4, seed=41)
    src = _random_state(L, 0.6, seed=lam)
    dst, acc = O.ne_tiles_launch(p, src, 9)
    changed = (dst & 1) != (src & 1)
    # each change toggles a site: the count has the parity of the sites that differ
    assert acc >= changed.sum() and (acc - changed.sum()) % 2 == 0
    # sites that changed carry the flag; the flag is never cleared
    assert np.all(dst[changed] & 2)
    assert np.all((dst & 2) >= (src & 2))
    assert np.array_equal(dst[~changed] & 1, src[~changed] & 1)
    # a site whose north or east neighbour is down at launch start and stays
    # down throughout cannot move: on an all-down lattice nothing happens
    zero = np.zeros((L, L), dtype=np.int8)
    dz, az = O.ne_tiles_launch(p, zero, 9)
    assert az == 0 and not dz.any()


def test_run_is_two_launches_per_sweep():
    L, B, lam = 32, 16, 16
    p = _params(L, B, lam, 0.3, seed=7)
    s = O.init_lattice(p)
    a, acc0 = O.ne_tiles_launch(p, s, 6)
    b, acc1 = O.ne_tiles_launch(p, a, 7)
    s2 = s.copy()
    rec = O.run(p, s2, 3, 1)
    np.testing.assert_array_equal(s2, b)
    bond, mag, unfl = O.recount(p, b)
    assert rec.tolist() == [[4, bond, mag, acc0 + acc1, unfl]]


def test_init_and_records_follow_ne_conventions():
    p = _params(64, 32, 16, 0.2, seed=13)
    q = O.Params(model=O.NORTH_EAST, dim=2, L=64, c=0.2, seed=13)
    np.testing.assert_array_equal(O.init_lattice(p), O.init_lattice(q))
    s = O.init_lattice(p)
    assert O.recount(p, s) == O.recount(q, s)


@pytest.mark.parametrize("L,B,lam", [(30, 8, 4), (32, 8, 3), (32, 1, 1)])
def test_invalid_parameters_rejected(L, B, lam):
    p = _params(L, B, lam, 0.3)
    s = np.zeros((L, L), dtype=np.int8)
    with pytest.raises(ValueError):
        O.ne_tiles_launch(p, s, 0)


# ---------------------------------------------------------------------------
# Balanced variant (end of Sec. 3.2): red then white sites, four launches per sweep.

TAG_NE_BALANCED = 3


def _bparams(L, B, lam, c, seed=1):
    return O.Params(model=O.NE_BALANCED, dim=2, L=L, c=c, seed=seed, tile=B, lam=lam)


def _predict_balanced_one_iteration(p, src, launch):
    """lambda = P/8: one iteration per launch; the red half reads src, the white
    half reads its own sub-lattice after the red half and the other
    sub-lattices as in src; lowest-numbered attempt wins."""
    L, B = p.L, p.tile
    P, lam = B * B, p.lam
    up_thr = O.threshold_from_prob(p.c / (1 - p.c))
    down_thr = O.threshold_from_prob((1 - p.c) / p.c)
    one = L == B
    cur = src.copy()
    flips = 0
    for h in range(2):
        n = cur & 1
        n0 = src & 1
        # neighbour inside the own sub-lattice (or B = L): current; else launch start
        north = np.where((np.arange(L) % B != 0)[:, None] | one, np.roll(n, 1, axis=0),
                         np.roll(n0, 1, axis=0))
        east = np.where((np.arange(L) % B != B - 1)[None, :] | one, np.roll(n, -1, axis=1),
                        np.roll(n0, -1, axis=1))
        nxt = cur.copy()
        for tau in range((L // B) ** 2):
            x0, y0 = (tau % (L // B)) * B, (tau // (L // B)) * B
            seen = set()
            for l in range(lam):
                a = h * lam + l
                w = O.philox4x32_10([tau, a // 2, launch, TAG_NE_BALANCED],
                                    [p.seed & 0xFFFFFFFF, p.seed >> 32])
                i = (w[2 * (a % 2)] * (P // 2)) >> 32
                if i in seen:
                    continue
                seen.add(i)
                r = i // (B // 2)
                cc = 2 * (i % (B // 2)) + ((r + h) & 1)
                y, x = y0 + r, x0 + cc
                assert (x + y) % 2 == h
                if not (north[y, x] and east[y, x]):
                    continue
                thr = down_thr if n[y, x] else up_thr
                if w[2 * (a % 2) + 1] < thr:
                    nxt[y, x] = ((cur[y, x] & 1) ^ 1) | 2
                    flips += 1
        cur = nxt
    return cur, flips


@pytest.mark.parametrize("L,B,c,launch", [(16, 8, 0.3, 5), (16, 4, 0.6, 0), (24, 8, 0.45, 77)])
def test_balanced_one_iteration_predicted_site_by_site(L, B, c, launch):
    p = _bparams(L, B, (B * B) // 8, c, seed=13)
    src = _random_state(L, 0.8, seed=L * B)
    dst, acc = O.ne_balanced_launch(p, src, launch)
    want, want_acc = _predict_balanced_one_iteration(p, src, launch)
    np.testing.assert_array_equal(dst, want)
    assert acc == want_acc


def test_balanced_keeps_the_product_measure():
    """Start from exact samples of Bernoulli(c)^N and apply one sweep (four
    launches): the up density and the north/east pair density stay c and c^2
    (the variant keeps the measure stationary), within 5 standard errors."""
    c, L = 0.42, 32
    dens, pairs = [], []
    for seed in range(40):
        p = _bparams(L, 8, 2, c, seed=1000 + seed)
        rng = np.random.default_rng(seed)
        s = np.ascontiguousarray((rng.random((L, L)) < c).astype(np.int8))
        O.run(p, s, seed, 1)
        n = s & 1
        dens.append(n.mean())
        pairs.append((n * np.roll(n, 1, axis=0)).mean() + (n * np.roll(n, -1, axis=1)).mean())
    N = L * L * len(dens)
    assert abs(np.mean(dens) - c) < 5 * math.sqrt(c * (1 - c) / N)
    assert abs(np.mean(pairs) / 2 - c * c) < 5 * math.sqrt(c * c * (1 - c * c) / N)


def test_balanced_launch_invariants_and_sweep():
    L, B, lam = 32, 8, 4
    p = _bparams(L, B, lam, 0.4, seed=43)
    src = _random_state(L, 0.6, seed=7)
    dst, acc = O.ne_balanced_launch(p, src, 9)
    changed = (dst & 1) != (src & 1)
    assert acc >= changed.sum() and (acc - changed.sum()) % 2 == 0
    assert np.all(dst[changed] & 2) and np.all((dst & 2) >= (src & 2))
    zero = np.zeros((L, L), dtype=np.int8)
    dz, az = O.ne_balanced_launch(p, zero, 9)
    assert az == 0 and not dz.any()
    # a sweep is launches 4t .. 4t+3, alternating the two copies
    s = O.init_lattice(p)
    cur, tot = s.copy(), 0
    for i in range(4):
        cur, a = O.ne_balanced_launch(p, cur, 4 * 5 + i)
        tot += a
    s2 = s.copy()
    rec = O.run(p, s2, 5, 1)
    np.testing.assert_array_equal(s2, cur)
    assert rec[0, 3] == tot and rec[0, 0] == 6
    # the balanced and the plain variant draw from different streams
    q = _params(L, B, lam, 0.4, seed=43)
    assert not np.array_equal(O.ne_tiles_launch(q, src, 9)[0], dst)


@pytest.mark.parametrize("L,B,lam", [(32, 8, 16), (32, 8, 3), (30, 10, 1)])
def test_balanced_invalid_parameters_rejected(L, B, lam):
    p = _bparams(L, B, lam, 0.3)
    with pytest.raises(ValueError):
        O.ne_balanced_launch(p, np.zeros((L, L), dtype=np.int8), 0)
