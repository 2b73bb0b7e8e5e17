"""Sweep indices at the top of their range: every schedule, the batched
kernels and both NE sub-lattice algorithms, started from a buffer with t0 just
below the limit of the 32-bit counter word (2^32 for the checkerboard sweep,
2^31 and 2^30 for the sub-lattice algorithms with two and four launches per
sweep), must equal the oracle run from the same state and t0 bit for bit, up
to the last allowed sweep; one sweep more is refused."""
import numpy as np
import pytest
import torch

import paper_1209_0296_amd as S
from helpers import expected_supported, run_oracle
from workloads import random_lattice

pytestmark = pytest.mark.gpu

T_END = 2 ** 32

SCHEDULES = [(S.MODE_SIMPLE, 0, 0), (S.MODE_HALF, 4, 1), (S.MODE_HALF, 3, 2), (S.MODE_FUSED, 4, 1),
             (S.MODE_FUSED, 5, 2), (S.MODE_HALF_WINDOW, 0, 0), (S.MODE_FUSED_WINDOW, 3, 0),
             (S.MODE_RESIDENT, 0, 0), (S.MODE_HALF_ROWS, 3, 2), (S.MODE_HALF_ROWS, 0, 4), (S.MODE_FUSED, 8, 4), (S.MODE_FUSED, 16, 2), (S.MODE_FUSED, 32, 4),
             (S.MODE_AUTO, 0, 0)]

SHAPES = [dict(L=64, T=2.269), dict(L=256, T=2.0), dict(L=40, two_s=2, T=1.5),
          dict(dim=3, L=16, T=4.5), dict(dim=3, L=32, two_s=2, T=3.0),
          dict(model=S.NORTH_EAST, L=64, c=0.3), dict(model=S.NE_COUPLED, L=64, J=1.0, h=0.1, T=2.2, c=0.5)]


def _start(sp):
    return random_lattice(sp.shape, two_s=sp.two_s, seed=sp.seed, model=sp.model, flag_fraction=0.2)


def _params(shape):
    return S.Params(init=S.INIT_BUFFER, t0=T_END - 8, seed=40 + shape, record_capacity=16, **SHAPES[shape])


# every (shape, schedule) pair the library offers; refusals are checked by the
# parity tests
CASES = [(i, launch) for i in range(len(SHAPES)) for launch in SCHEDULES
         if expected_supported(_params(i), launch)]


@pytest.mark.parametrize("shape,launch", CASES)
def test_last_sweep_indices(shape, launch):
    n = 8
    sp = _params(shape)
    print(f"case large t shape={SHAPES[shape]} launch={launch}", flush=True)
    start = _start(sp)
    lat = S.Lattice(sp, init_spins=torch.from_numpy(start))
    lat.set_launch(*launch)
    recs = [S.records_to_array(lat.measure())]
    lat.sweep(3)
    recs.append(S.records_to_array(lat.measure()))
    lat.sweep(n - 3)
    recs.append(S.records_to_array(lat.measure()))
    with pytest.raises(S.SpinlatError) as e:
        lat.sweep(1)
    assert e.value.status == 6
    g_s = lat.spins()
    lat.close()
    o_s, o_r = run_oracle(sp, n, start=start)
    g_r = np.vstack(recs)
    assert g_r[-1, 0] == T_END
    np.testing.assert_array_equal(g_r, o_r)
    np.testing.assert_array_equal(g_s, o_s)


@pytest.mark.parametrize("model,limit", [(S.NE_SUBLATTICE, 2 ** 31), (S.NE_SUBLATTICE_BALANCED, 2 ** 30)])
def test_sub_lattice_last_sweep_indices(model, limit):
    n = 4
    sp = S.Params(model=model, L=64, c=0.3, init=S.INIT_BUFFER, t0=limit - n, seed=9, ne_side=16,
                  ne_lambda=8, record_capacity=8)
    start = _start(sp)
    lat = S.Lattice(sp, init_spins=torch.from_numpy(start))
    recs = [S.records_to_array(lat.measure())]
    lat.sweep(n)
    recs.append(S.records_to_array(lat.measure()))
    with pytest.raises(S.SpinlatError) as e:
        lat.sweep(1)
    assert e.value.status == 6
    g_s = lat.spins()
    lat.close()
    o_s, o_r = run_oracle(sp, n, start=start)
    np.testing.assert_array_equal(np.vstack(recs), o_r)
    np.testing.assert_array_equal(g_s, o_s)


def test_batched_last_sweep_indices():
    """Jobs of every batched class with t0 = 2^32 - 8 run their last 8 sweeps
    in one batch; a job asking for one sweep more is refused."""
    n = 8
    shapes = [dict(L=64, T=2.269), dict(L=1040, T=2.3), dict(L=40, two_s=2, T=1.5), dict(dim=3, L=16, T=4.5),
              dict(dim=3, L=24, two_s=2, T=3.0), dict(model=S.NORTH_EAST, L=64, c=0.3),
              dict(model=S.NE_COUPLED, L=64, J=1.0, h=0.1, T=2.2, c=0.5), dict(L=64, T=0.05)]
    b = S.Batch(64 << 20, max_jobs=16, record_capacity=n + 1)
    jobs = {}
    for i, kw in enumerate(shapes):
        sp = S.Params(init=S.INIT_BUFFER, t0=T_END - n, seed=70 + i, **kw)
        start = _start(sp)
        jobs[b.add(sp, n, init_spins=torch.from_numpy(start))] = (sp, start)
    sp0 = S.Params(init=S.INIT_BUFFER, t0=T_END - n, seed=1, L=64)
    with pytest.raises(S.SpinlatError) as e:
        b.add(sp0, n + 1, init_spins=torch.from_numpy(_start(sp0)))
    assert e.value.status == 6
    with pytest.raises(S.SpinlatError) as e:
        b.add(sp0, 2 ** 64 - 1, init_spins=torch.from_numpy(_start(sp0)))
    assert e.value.status == 6
    got = {j: [] for j in jobs}
    while any(b.status(j)[1] for j in jobs):
        b.sweep(3)
        for j, r in b.drain().items():
            got[j].append(r)
    for j, r in b.drain().items():
        got[j].append(r)
    for j, (sp, start) in jobs.items():
        o_s, o_r = run_oracle(sp, n, start=start)
        np.testing.assert_array_equal(np.vstack(got[j]), o_r)
        np.testing.assert_array_equal(b.spins(j), o_s)
    b.close()


def test_sweep_count_cannot_wrap():
    """sl_sweep(2^64 - 1) (what a negative count becomes in a C uint64) is
    refused with nothing enqueued, and the binding rejects negative counts."""
    import ctypes

    sp = S.Params(L=64, record_capacity=4)
    lat = S.Lattice(sp)
    st = S.lib().sl_sweep(lat._h, ctypes.c_uint64(2 ** 64 - 1))
    assert st == 5
    with pytest.raises(ValueError):
        lat.sweep(-1)
    assert lat.counts() == (1, 0)
    lat.close()
