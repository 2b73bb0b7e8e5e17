"""GPU parity of batched sweeps: every job of a mixed batch must reproduce,
bit for bit, the oracle run of the same job alone (lattice and every record),
whatever else shares its launches and whenever it was admitted."""
import numpy as np
import pytest

import paper_1209_0296_amd as S
from helpers import run_oracle

pytestmark = pytest.mark.gpu


def _mixed_jobs():
    jobs = [
        S.Params(L=64, T=2.269, init=S.INIT_COLD, seed=1),
        S.Params(L=40, T=2.0, seed=2),                      # D = 1 rows
        S.Params(L=136, two_s=2, T=1.7, seed=3),
        S.Params(L=256, T=2.4, h=0.1, seed=4),              # 32-word rows, D = 4
        S.Params(L=1024, T=2.269, seed=5),                  # 128-word rows, D = 2
        S.Params(dim=3, L=16, T=4.5, seed=6),
        S.Params(dim=3, L=24, two_s=2, T=3.2, seed=7),      # resident, else 3-word rows: 1 word per lane
        S.Params(dim=3, L=64, T=4.0, J=0.9, seed=8),
        S.Params(model=S.NORTH_EAST, L=72, c=0.2, seed=9),
        S.Params(model=S.NORTH_EAST, L=128, c=0.1, seed=10),
        S.Params(L=936, T=2.3, seed=11),                   # 117-word rows: window kernel
        S.Params(L=600, two_s=2, T=1.6, seed=16),          # 75-word rows: window kernel, spin-1
        S.Params(model=S.NORTH_EAST, L=936, c=0.2, seed=17),  # NE, 117-word rows: window kernel
        S.Params(L=64, T=0.05, seed=12),                   # zero thresholds: window kernel
        S.Params(dim=3, L=40, two_s=2, T=2.9, seed=13),     # 5-word rows: 1 word per lane
        S.Params(dim=3, L=56, T=4.4, seed=14),              # 7-word rows: 1 word per lane
        S.Params(dim=3, L=72, T=4.6, h=0.05, seed=15),      # 9-word rows: 1 word per lane
    ]
    return jobs


def _check_job(batch, jid, sp, recs, nsweeps):
    o_s, o_r = run_oracle(sp, nsweeps)
    np.testing.assert_array_equal(np.vstack(recs), o_r)
    np.testing.assert_array_equal(batch.spins(jid), o_s)


FLAGS = [0, S.BATCH_NO_GRAPH, S.BATCH_NO_FUSED | S.BATCH_NO_RESIDENT,
         S.BATCH_NO_GRAPH | S.BATCH_NO_FUSED | S.BATCH_NO_RESIDENT]


@pytest.mark.parametrize("flags", FLAGS)
def test_mixed_batch_matches_each_job_alone(flags):
    """Every class (resident, fused, row groups, walks, windows), with and
    without graph replay."""
    print(f"case mixed batch flags={flags}", flush=True)
    jobs = _mixed_jobs()
    b = S.Batch(arena_bytes=96 << 20, max_jobs=24, record_capacity=64, flags=flags)
    ids = [b.add(p, sweeps=12) for p in jobs]
    assert all(i is not None for i in ids)
    recs = {i: [S.records_to_array(b.measure(i))] for i in ids}
    b.sweep(5)
    for i in ids:
        recs[i].append(S.records_to_array(b.measure(i)))
    b.sweep(100)  # every job stops at its own 12
    for i, p in zip(ids, jobs):
        assert b.status(i)[:2] == (12, 0)
        recs[i].append(S.records_to_array(b.measure(i)))
        _check_job(b, i, p, recs[i], 12)
    b.close()


def test_coupled_ne_jobs_in_a_mixed_batch():
    """Coupled NE jobs (rows within one wave) share launches with Ising and
    J = 0 NE jobs and still equal the oracle run of each job alone."""
    jobs = [
        S.Params(model=S.NE_COUPLED, L=64, J=1.0, h=0.2, T=2.0, c=0.6, seed=31),
        S.Params(model=S.NE_COUPLED, L=40, J=-0.5, h=0.0, T=1.5, c=0.4, seed=32),   # D = 1 rows
        S.Params(model=S.NE_COUPLED, L=512, J=1.0, h=-0.1, T=2.5, c=0.5, seed=33),  # D = 4 rows
        S.Params(model=S.NORTH_EAST, L=64, c=0.2, seed=34),
        S.Params(L=64, T=2.269, seed=35),
        S.Params(L=936, T=2.3, seed=36),                                            # window kernel
    ]
    b = S.Batch(arena_bytes=32 << 20, max_jobs=8, record_capacity=32)
    ids = [b.add(p, sweeps=20) for p in jobs]
    recs = {i: [S.records_to_array(b.measure(i))] for i in ids}
    b.sweep(9)
    for i in ids:
        recs[i].append(S.records_to_array(b.measure(i)))
    b.sweep(50)
    for i, p in zip(ids, jobs):
        print(f"case batch coupled job {i} model={p.model} L={p.L}", flush=True)
        assert b.status(i)[:2] == (20, 0)
        recs[i].append(S.records_to_array(b.measure(i)))
        _check_job(b, i, p, recs[i], 20)
    b.close()


def test_uneven_budgets_and_late_admission():
    b = S.Batch(arena_bytes=32 << 20, max_jobs=8, record_capacity=16)
    early = S.Params(L=128, T=2.3, seed=21)
    ja = b.add(early, sweeps=30)
    ra = [S.records_to_array(b.measure(ja))]
    b.sweep(7)
    late = S.Params(dim=3, L=32, two_s=2, T=3.0, seed=22)
    jb = b.add(late, sweeps=9)
    short = S.Params(L=64, T=1.9, seed=23)
    jc = b.add(short, sweeps=3)
    rb = [S.records_to_array(b.measure(jb))]
    rc = [S.records_to_array(b.measure(jc))]
    # the ring holds 16 records: sweep in chunks and drain between them
    while any(b.status(j)[1] for j in (ja, jb, jc)):
        b.sweep(10)
        ra.append(S.records_to_array(b.measure(ja)))
        rb.append(S.records_to_array(b.measure(jb)))
        rc.append(S.records_to_array(b.measure(jc)))
    _check_job(b, ja, early, ra, 30)
    _check_job(b, jb, late, rb, 9)
    _check_job(b, jc, short, rc, 3)
    b.close()


def test_admission_by_footprint_and_reuse():
    cfg = S.batch_config(max_jobs=8, record_capacity=8)
    p = S.Params(L=512, T=2.2, seed=31)
    need = S.batch_job_bytes(p, cfg)
    base = S.batch_base_bytes(cfg)
    b = S.Batch(arena_bytes=base + 2 * need + 4096, max_jobs=8, record_capacity=8)
    j1 = b.add(p, sweeps=4)
    j2 = b.add(S.Params(L=512, T=2.5, seed=32), sweeps=4)
    assert j1 is not None and j2 is not None
    assert b.add(S.Params(L=512, T=2.0, seed=33), sweeps=4) is None  # no room: refused
    r1 = [S.records_to_array(b.measure(j1))]
    b.sweep(4)
    r1.append(S.records_to_array(b.measure(j1)))
    _check_job(b, j1, p, r1, 4)
    b.remove(j1)
    p3 = S.Params(L=512, T=2.0, seed=33)
    j3 = b.add(p3, sweeps=4)  # fits again in the freed space
    assert j3 is not None
    r3 = [S.records_to_array(b.measure(j3))]
    b.sweep(4)
    r3.append(S.records_to_array(b.measure(j3)))
    _check_job(b, j3, p3, r3, 4)
    b.close()


def test_batch_equals_standalone_lattice():
    """Batched and standalone GPU runs of the same job agree (and with the oracle)."""
    from helpers import run_gpu

    p = S.Params(L=256, T=2.269, seed=41, record_capacity=32)
    g_s, g_r = run_gpu(p, 20)
    b = S.Batch(arena_bytes=48 << 20, max_jobs=4, record_capacity=32)
    j = b.add(p, sweeps=20)
    r = [S.records_to_array(b.measure(j))]
    b.sweep(20)
    r.append(S.records_to_array(b.measure(j)))
    np.testing.assert_array_equal(np.vstack(r), g_r)
    np.testing.assert_array_equal(b.spins(j), g_s)
    b.close()


@pytest.mark.parametrize("flags", FLAGS)
def test_drain_collects_every_job(flags):
    """sl_batch_drain (one fold launch, one copy) gives each job's records; the
    chunks of 7 sweeps flip the fused jobs' current copy every call."""
    print(f"case drain flags={flags}", flush=True)
    jobs = _mixed_jobs()
    b = S.Batch(arena_bytes=96 << 20, max_jobs=24, record_capacity=8, flags=flags)
    ids = [b.add(p, sweeps=10 + k) for k, p in enumerate(jobs)]
    recs = {i: [] for i in ids}
    while True:
        got = b.drain()
        for j, r in got.items():
            recs[j].append(r)
        if not any(b.status(i)[1] for i in ids):
            break
        b.sweep(7)
    for i, p in zip(ids, jobs):
        _check_job(b, i, p, recs[i], b.status(i)[0])
    b.close()


def test_graph_replay_across_changing_mixes():
    """Jobs join and leave between calls of the same shape (the captured graph
    is replayed with other work lists); lattices are read mid-run, between
    calls of odd length, from the fused jobs' alternating copies."""
    b = S.Batch(arena_bytes=128 << 20, max_jobs=32, record_capacity=16)
    live = {}
    specs = [S.Params(L=L, T=2.0 + 0.01 * k, seed=200 + k, two_s=1 + (k % 2), dim=2 if k % 3 else 3)
             for k, L in enumerate([64, 128, 256, 512, 48, 96, 32, 160, 64, 128, 256, 80])]
    specs = [S.Params(**{**p.__dict__, "L": min(p.L, 64) if p.dim == 3 else p.L}) for p in specs]
    rounds = 0
    pending = list(range(len(specs)))
    while pending or live:
        while pending and len(live) < 6:
            k = pending.pop(0)
            j = b.add(specs[k], sweeps=9 + 4 * (k % 3))
            live[j] = (k, [S.records_to_array(b.measure(j))])
        b.sweep(5)
        rounds += 1
        for j, (k, recs) in list(live.items()):
            recs.append(S.records_to_array(b.measure(j)))
            done, remaining, _ = b.status(j)
            if rounds % 2 == 1 or remaining == 0:
                o_s, o_r = run_oracle(specs[k], done)
                np.testing.assert_array_equal(np.vstack(recs), o_r)
                np.testing.assert_array_equal(b.spins(j), o_s)
            if remaining == 0:
                b.remove(j)
                del live[j]
    b.close()


def test_job_table_full_is_not_an_error():
    """With max_jobs below what the arena holds, add() returns None when the
    table is full, and the server queues the request until a slot frees."""
    from paper_1209_0296_amd.serve import Request, Server

    b = S.Batch(arena_bytes=64 << 20, max_jobs=2, record_capacity=8)
    assert b.add(S.Params(L=64, seed=1), 4) is not None
    assert b.add(S.Params(L=64, seed=2), 4) is not None
    assert b.add(S.Params(L=64, seed=3), 4) is None
    b.close()
    reqs = [Request(i, 0.0, S.Params(L=64 if i % 2 else 128, T=2.2, seed=300 + i), 10 + i) for i in range(9)]
    srv = Server(64 << 20, max_jobs=3, chunk=4)
    outcomes, stats = srv.run(reqs, realtime=False)
    srv.close()
    assert stats["jobs"] == len(reqs)
    for r in reqs:
        np.testing.assert_array_equal(outcomes[r.id].records, run_oracle(r.params, r.sweeps)[1])


def test_graph_cache_eviction_keeps_results():
    """More call shapes than the graph cache holds (sweeps per call 1 .. 24 on
    every family, both streams): evicted graphs are rebuilt and every job still
    equals the oracle run alone."""
    jobs = [S.Params(dim=3, L=32, T=4.5, seed=401),              # row groups, spin-1/2
            S.Params(dim=3, L=40, two_s=2, T=3.0, seed=402),     # row groups, spin-1
            S.Params(L=512, T=2.3, seed=403),                    # fused
            S.Params(model=S.NORTH_EAST, L=936, c=0.3, seed=404),  # column windows
            S.Params(L=64, T=2.0, seed=405)]                     # resident
    total = sum(range(1, 25))
    b = S.Batch(arena_bytes=96 << 20, max_jobs=8, record_capacity=32)
    ids = [b.add(p, sweeps=total) for p in jobs]
    recs = {i: [] for i in ids}
    for n in range(1, 25):
        b.sweep(n)
        for j, r in b.drain().items():
            recs[j].append(r)
    for i, p in zip(ids, jobs):
        print(f"case eviction job {i} L={p.L} dim={p.dim}", flush=True)
        assert b.status(i)[:2] == (total, 0)
        _check_job(b, i, p, recs[i], total)
    b.close()
