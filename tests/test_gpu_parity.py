"""GPU parity: every launch schedule of the HIP sweep must reproduce the
oracle's lattice and every per-sweep record bit for bit (integer result:
exact equality), on small lattices spanning several windows, strips and a
ragged tail, at the benchmarked sizes, and across split runs and restarts."""
import numpy as np
import pytest

import paper_1209_0296_amd as S
from helpers import assert_refused, expected_supported, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

SIMPLE = (S.MODE_SIMPLE, 0, 0)
HALF = (S.MODE_HALF, 0, 0)
FUSED = (S.MODE_FUSED, 0, 0)
HALF_W = (S.MODE_HALF_WINDOW, 0, 0)
FUSED_W = (S.MODE_FUSED_WINDOW, 0, 0)
AUTO = (S.MODE_AUTO, 0, 0)
RESIDENT = (S.MODE_RESIDENT, 0, 0)
# whole-row kernels: (mode, rows per strip, words per lane)
ROW = [(m, H, D) for m in (S.MODE_HALF, S.MODE_FUSED) for H, D in ((3, 1), (8, 2), (5, 4))]
# whole-row walks with the unrolled strip heights, and row groups without a walk
ROW += [(S.MODE_FUSED, 2, 4), (S.MODE_FUSED, 4, 2), (S.MODE_FUSED, 8, 4), (S.MODE_FUSED, 16, 2), (S.MODE_FUSED, 32, 4), (S.MODE_HALF_ROWS, 0, 0),
        (S.MODE_HALF_ROWS, 1, 1), (S.MODE_HALF_ROWS, 3, 2), (S.MODE_HALF_ROWS, 16, 4)]


def _check(sp, nsweeps, launch=None, chunks=None, nthreads=0):
    print(f"case model={sp.model} dim={sp.dim} L={sp.L} two_s={sp.two_s} T={sp.T} c={sp.c} "
          f"n={nsweeps} launch={launch} chunks={chunks}", flush=True)
    if launch is not None and not expected_supported(sp, launch):
        assert_refused(sp, launch)
        return None
    g_s, g_r = run_gpu(sp, nsweeps, launch=launch, chunks=chunks)
    o_s, o_r = run_oracle(sp, nsweeps, nthreads=nthreads)
    assert g_r.shape == o_r.shape
    np.testing.assert_array_equal(g_r, o_r)
    np.testing.assert_array_equal(g_s, o_s)


@pytest.mark.parametrize("launch", [SIMPLE, HALF, FUSED, HALF_W, FUSED_W, RESIDENT, AUTO])
def test_ising2d_L64_cold_1000_sweeps(launch):
    """64x64, J=1, T=2.269, cold start, seed 1, 1000 sweeps, every record."""
    sp = S.Params(L=64, T=2.269, init=S.INIT_COLD, seed=1, record_capacity=1001)
    _check(sp, 1000, launch=launch)


# Colour rows of L/8 words.  Window kernels: L = 8, 16, 64 one group per row;
# 40, 72, 136 windows with wrapped columns; 512 exactly 64 columns; 1040
# three windows with a ragged tail.  Row kernels: row groups of 1..64 lanes,
# and of 128 or 256 lanes (several waves exchanging edge words) at L = 1024
# and 2048; L = 1040 fits no row group.
SHAPES_2D = [8, 16, 40, 64, 72, 136, 512, 1024, 1040, 2048]


@pytest.mark.parametrize("L", SHAPES_2D)
@pytest.mark.parametrize("two_s", [1, 2])
@pytest.mark.parametrize("launch", [SIMPLE, HALF_W, FUSED_W, RESIDENT, AUTO] + ROW)
def test_ising2d_shapes(L, two_s, launch):
    n = 12 if L >= 512 else 25
    sp = S.Params(L=L, two_s=two_s, T=2.0 if two_s == 1 else 1.5, seed=7 + L, record_capacity=64)
    _check(sp, n, launch=launch)


@pytest.mark.parametrize("rows", [1, 2, 3, 7, 16, 33])
@pytest.mark.parametrize("mode", [S.MODE_HALF_WINDOW, S.MODE_FUSED_WINDOW, S.MODE_HALF,
                                  S.MODE_FUSED])
def test_strip_heights(rows, mode):
    sp = S.Params(L=136, T=2.269, seed=5, record_capacity=64)
    words = 1 if mode in (S.MODE_HALF, S.MODE_FUSED) else 0
    _check(sp, 10, launch=(mode, rows, words))


@pytest.mark.parametrize("L", [8, 16, 24, 40, 64, 128])
@pytest.mark.parametrize("two_s", [1, 2])
@pytest.mark.parametrize("launch", [SIMPLE, HALF_W, (S.MODE_HALF_WINDOW, 5, 0), AUTO, RESIDENT,
                                    (S.MODE_HALF, 3, 1), (S.MODE_HALF, 8, 2), (S.MODE_HALF, 4, 4),
                                    (S.MODE_HALF_ROWS, 1, 1), (S.MODE_HALF_ROWS, 3, 2),
                                    (S.MODE_HALF_ROWS, 0, 4), (S.MODE_HALF_ROWS, 16, 4)])
def test_ising3d_shapes(L, two_s, launch):
    sp = S.Params(dim=3, L=L, two_s=two_s, T=4.5 if two_s == 1 else 3.2, seed=3 + L,
                  record_capacity=64)
    _check(sp, 12, launch=launch)


# Ragged row groups: colour rows of L/8 words that 2 or 4 words per lane do
# not divide (L % 16 = 8 or L % 32 in {8, 16, 24}); the last lane holds the
# row's last D words, some of which lane R-2 also holds.  Row groups of 2 to
# 33 lanes, the duplicated words in both lane orders (row parity 0 and 1).
RAGGED_3D = [24, 40, 56, 72, 88, 120, 136]
RAGGED_2D = [24, 40, 72, 200, 1032]
RAGGED_LAUNCH = [(S.MODE_HALF_ROWS, 4, 2), (S.MODE_HALF_ROWS, 4, 4), (S.MODE_HALF_ROWS, 8, 4),
                 (S.MODE_HALF_ROWS, 1, 2), (S.MODE_HALF_ROWS, 0, 0), AUTO]


@pytest.mark.parametrize("L", RAGGED_3D)
@pytest.mark.parametrize("two_s", [1, 2])
@pytest.mark.parametrize("launch", RAGGED_LAUNCH)
def test_ising3d_ragged_rows(L, two_s, launch):
    sp = S.Params(dim=3, L=L, two_s=two_s, T=4.4 if two_s == 1 else 3.1, h=0.03 * (L % 3),
                  seed=300 + L, record_capacity=64)
    _check(sp, 9, launch=launch)


@pytest.mark.parametrize("L", RAGGED_2D)
@pytest.mark.parametrize("two_s", [1, 2])
@pytest.mark.parametrize("launch", RAGGED_LAUNCH)
def test_ising2d_ragged_rows(L, two_s, launch):
    sp = S.Params(L=L, two_s=two_s, T=2.2 if two_s == 1 else 1.6, seed=400 + L, record_capacity=64)
    _check(sp, 15, launch=launch)


def test_ragged_rows_refused_for_ne():
    """NE lattices keep rows that the words per lane divide."""
    for launch in ((S.MODE_HALF_ROWS, 4, 2), (S.MODE_HALF_ROWS, 4, 4)):
        assert_refused(S.Params(model=S.NORTH_EAST, L=40, c=0.2, seed=1), launch)
        assert_refused(S.Params(model=S.NE_COUPLED, L=40, J=1.0, T=2.0, c=0.3, seed=1), launch)


@pytest.mark.parametrize("L", [8, 32, 72, 1040, 2048])
@pytest.mark.parametrize("c", [0.05, 0.2, 0.6])
@pytest.mark.parametrize("launch", [SIMPLE, HALF_W, FUSED_W, RESIDENT, AUTO] + ROW)
def test_ne_shapes(L, c, launch):
    sp = S.Params(model=S.NORTH_EAST, L=L, c=c, seed=11, record_capacity=64)
    _check(sp, 12 if L > 512 else 30, launch=launch)


def test_resident_chunks_and_mixed_modes():
    """More sweeps than one resident launch runs (4096), then a switch to the
    fused mode and back, on an 8x8 and a 48x48 lattice."""
    sp = S.Params(L=8, T=2.269, seed=21, record_capacity=5001)
    _check(sp, 5000, launch=RESIDENT)
    sp = S.Params(L=48, two_s=2, T=1.7, seed=22, record_capacity=64)
    o_s, o_r = run_oracle(sp, 30)
    import paper_1209_0296_amd as P

    lat = P.Lattice(sp)
    recs = [P.records_to_array(lat.measure())]
    for mode, n in ((RESIDENT, 7), (FUSED, 5), (RESIDENT, 18)):
        lat.set_launch(*mode)
        lat.sweep(n)
        recs.append(P.records_to_array(lat.measure()))
    np.testing.assert_array_equal(np.vstack(recs), o_r)
    np.testing.assert_array_equal(lat.spins(), o_s)
    lat.close()


@pytest.mark.parametrize("kw", [dict(L=216, T=2.3), dict(dim=3, L=32, two_s=2, T=3.0),
                                dict(model=S.NORTH_EAST, L=216, c=0.35)])
def test_resident_largest_lattices(kw):
    """The largest lattices under the 48 KiB limit with L % 8 == 0: 2D L = 216
    (46656 sites), 3D L = 32 (32768 sites)."""
    sp = S.Params(seed=31, record_capacity=32, **kw)
    _check(sp, 20, launch=RESIDENT)


@pytest.mark.parametrize("kw", [dict(L=224), dict(L=256), dict(dim=3, L=40)])
def test_resident_refuses_large_lattices(kw):
    lat = S.Lattice(S.Params(seed=1, **kw))
    with pytest.raises(S.SpinlatError):
        lat.set_launch(*RESIDENT)
    lat.close()


def test_zero_threshold_tables_use_window_kernels():
    """At tiny T some thresholds are 0 (never accept); the 32-bit table of the
    row kernels cannot hold them, so AUTO picks the window kernels."""
    for dim in (2, 3):
        sp = S.Params(dim=dim, L=64 if dim == 2 else 16, T=0.05, seed=9, record_capacity=16)
        assert 0 in S.threshold_table(sp)
        _check(sp, 5, launch=AUTO)
        with pytest.raises(S.SpinlatError):
            lat = S.Lattice(sp)
            try:
                lat.set_launch(S.MODE_HALF, 8, 2)
            finally:
                lat.close()


def test_fields_and_couplings():
    for kw in (dict(T=1.3, h=0.37), dict(T=2.1, J=-1.0, h=0.2), dict(two_s=2, T=1.1, h=-0.3),
               dict(dim=3, T=3.0, h=0.5), dict(dim=3, two_s=2, T=2.0, J=0.7, h=-0.2)):
        for launch in (HALF, FUSED, HALF_W, FUSED_W) if kw.get("dim", 2) == 2 else (HALF, HALF_W):
            sp = S.Params(L=40, seed=13, record_capacity=64, **kw)
            _check(sp, 10, launch=launch)


def test_infinite_temperature_flips_everything():
    sp = S.Params(L=64, T=float("inf"), seed=2, record_capacity=8)
    for launch in (SIMPLE, HALF, FUSED, HALF_W, FUSED_W):
        g_s, g_r = run_gpu(sp, 2, launch=launch)
        o_s, o_r = run_oracle(sp, 2)
        np.testing.assert_array_equal(g_s, o_s)
        np.testing.assert_array_equal(g_r, o_r)
        assert np.all(g_r[1:, 3] == sp.nsites)


def test_split_runs_and_mixed_schedules():
    """sweep(a) + sweep(b) + ... with different schedules == one run."""
    import torch

    sp = S.Params(L=136, T=2.269, seed=21, record_capacity=64)  # noqa
    lat = S.Lattice(sp)
    recs = [S.records_to_array(lat.measure())]
    for launch, n in ((SIMPLE, 3), (FUSED, 4), (HALF, 2), ((S.MODE_FUSED_WINDOW, 5, 0), 5), (HALF_W, 1),
                      ((S.MODE_FUSED, 3, 1), 3), ((S.MODE_HALF, 2, 1), 2)):
        lat.set_launch(*launch)
        lat.sweep(n)
        if n > 2:
            recs.append(S.records_to_array(lat.measure()))
    recs.append(S.records_to_array(lat.measure()))
    g_s = lat.spins()
    lat.close()
    o_s, o_r = run_oracle(sp, 20)
    np.testing.assert_array_equal(np.vstack(recs), o_r)
    np.testing.assert_array_equal(g_s, o_s)


@pytest.mark.parametrize("model,dim,two_s", [(0, 2, 1), (0, 3, 2), (1, 2, 1), (4, 2, 1)])
def test_checkpoint_restart(model, dim, two_s):
    """copy_spins at sweep a, recreate from that buffer with t0 = a, continue:
    identical to the uninterrupted run (the random numbers carry no state)."""
    L = 40 if dim == 3 else 72
    base = dict(model=model, dim=dim, L=L, two_s=two_s, T=2.5, c=0.3, seed=17, record_capacity=64)
    sp = S.Params(**base)
    lat = S.Lattice(sp)
    lat.sweep(7)
    lat.measure()
    snap = lat.copy_spins().clone()
    lat.close()
    sp2 = S.Params(**base, init=S.INIT_BUFFER, t0=7)
    lat2 = S.Lattice(sp2, init_spins=snap)
    r0 = S.records_to_array(lat2.measure())
    lat2.sweep(5)
    r = S.records_to_array(lat2.measure())
    g_s = lat2.spins()
    lat2.close()
    o_s, o_r = run_oracle(sp, 12)
    np.testing.assert_array_equal(g_s, o_s)
    np.testing.assert_array_equal(r, o_r[8:])
    assert r0[0, 0] == 7
    np.testing.assert_array_equal(r0[0, 1:3], o_r[7, 1:3])


def test_buffer_init_roundtrip():
    import torch
    from workloads import random_lattice

    for kw in (dict(L=64), dict(L=40, two_s=2), dict(dim=3, L=16), dict(model=1, L=64, c=0.3),
               dict(model=4, L=64, J=1.0, h=0.2, T=2.0, c=0.5), dict(model=4, L=256, J=-0.5, T=1.5)):
        sp = S.Params(init=S.INIT_BUFFER, seed=3, record_capacity=8, **kw)
        start = random_lattice(sp.shape, two_s=sp.two_s, seed=5, model=sp.model,
                               flag_fraction=0.3)
        lat = S.Lattice(sp, init_spins=torch.from_numpy(start))
        np.testing.assert_array_equal(lat.spins(), start)
        lat.sweep(3)
        recs = S.records_to_array(lat.measure())
        g = lat.spins()
        lat.close()
        o_s, o_r = run_oracle(sp, 3, start=start)
        np.testing.assert_array_equal(g, o_s)
        np.testing.assert_array_equal(recs, o_r)


def test_ne_persistence_reset():
    sp = S.Params(model=S.NORTH_EAST, L=64, c=0.2, seed=4, record_capacity=64)
    lat = S.Lattice(sp)
    lat.sweep(10)
    r1 = S.records_to_array(lat.measure())
    lat.reset_persistence()
    lat.sweep(5)
    r2 = S.records_to_array(lat.measure())
    spins = lat.spins()
    lat.close()
    assert np.all(np.diff(r1[:, 4]) <= 0) and r1[0, 4] == sp.nsites
    assert np.all(np.diff(r2[:, 4]) <= 0)
    import oracle as O
    from helpers import oracle_params

    op = oracle_params(sp)
    s = O.init_lattice(op)
    O.run(op, s, 0, 10, records=False)
    O.reset_persistence(op, s)
    rec = O.run(op, s, 10, 5)
    np.testing.assert_array_equal(r2, rec)
    np.testing.assert_array_equal(spins, s)


def test_record_ring_errors():
    sp = S.Params(L=64, record_capacity=4)
    lat = S.Lattice(sp)
    lat.sweep(3)
    with pytest.raises(S.SpinlatError) as e:
        lat.sweep(1)
    assert e.value.status == 5
    recs = lat.measure()
    assert len(recs) == 4 and list(recs["t"]) == [0, 1, 2, 3]
    lat.sweep(4)
    assert len(lat.measure()) == 4
    lat.close()
    sp = S.Params(L=64, t0=2 ** 32 - 2, record_capacity=8)
    lat = S.Lattice(sp)
    lat.sweep(2)
    with pytest.raises(S.SpinlatError) as e:
        lat.sweep(1)
    assert e.value.status == 6
    lat.close()


# ---------------------------------------------------------------------------
# Benchmarked sizes, in the schedule bench.py times (AUTO), against the oracle
# on all host threads: the whole lattice and every record.

@pytest.mark.parametrize("name,nsweeps", [("ising2d_L8192", 3), ("ising3d_L256_s12", 4),
                                          ("ising3d_L256_s1", 3), ("ne2d_L4096", 6),
                                          ("ne2d_coupled_L4096", 4)])
def test_benchmarked_sizes(name, nsweeps):
    from workloads import CONFIGS

    cfg = CONFIGS[name]
    sp = S.Params(model=cfg["model"], dim=cfg["dim"], L=cfg["L"], two_s=cfg["two_s"],
                  J=cfg.get("J", 1.0), h=cfg.get("h", 0.0), T=cfg.get("T", 1.0),
                  c=cfg.get("c", 0.1), seed=cfg["seed"], init=cfg["init"], record_capacity=16)
    _check(sp, nsweeps, launch=AUTO, nthreads=16)


def test_out_of_cache_size():
    """2D L = 32768 (1 GiB per copy, 2 GiB buffer; byte offsets past 2^31): one
    sweep in the benchmarked schedule, whole lattice and records."""
    sp = S.Params(L=32768, T=2.269, seed=1, record_capacity=4)
    _check(sp, 1, launch=AUTO, nthreads=16)


@pytest.mark.parametrize("T", [2.0, 2.6])
def test_ising2d_L8192_other_temperatures(T):
    sp = S.Params(L=8192, T=T, seed=1, record_capacity=8)
    _check(sp, 2, launch=AUTO, nthreads=16)


def test_zero_sweeps_and_single_record_ring():
    """sweep(0) is a no-op; a ring of one record holds r_0 only, so a sweep
    fails until it is drained, then each sweep fits exactly."""
    sp = S.Params(L=64, T=2.0, seed=8, record_capacity=1)
    o_s, o_r = run_oracle(sp, 3)
    lat = S.Lattice(sp)
    lat.sweep(0)
    with pytest.raises(S.SpinlatError):
        lat.sweep(1)
    recs = [S.records_to_array(lat.measure())]
    for _ in range(3):
        lat.sweep(1)
        recs.append(S.records_to_array(lat.measure()))
    np.testing.assert_array_equal(np.vstack(recs), o_r)
    np.testing.assert_array_equal(lat.spins(), o_s)
    lat.close()


@pytest.mark.parametrize("kw", [dict(L=8192, two_s=2, T=1.6935),     # spin-1: 16-row strips, 2 words
                                dict(L=16384, T=2.269),               # spin-1/2: 32-row strips, 4 words
                                dict(model=S.NORTH_EAST, L=8192, c=0.1)])
def test_large_default_schedules(kw):
    """The default schedules of the large 2D shapes, whole lattice and records."""
    sp = S.Params(seed=7, record_capacity=4, **kw)
    _check(sp, 2, launch=AUTO, nthreads=16)
