"""sl_sweep_static (the entry point that allocates nothing) against the
lattice entry points it stands for: create + sweep(n) + measure + copy_spins
must give the same lattice and records bit for bit, on two calls in a row
(the second on a smaller lattice, so stale working memory would show), and a
lattice beyond the static working memory is refused."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1209_0296_amd as S

pytestmark = pytest.mark.gpu


def _static(sp, n):
    spins = torch.empty(sp.nsites, dtype=torch.int8, device="cuda")
    recs = torch.empty((n + 1) * 5, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    cp = sp.c_struct()
    st = S.lib().sl_sweep_static(ctypes.byref(cp), n, spins.data_ptr(), recs.data_ptr(), stream.cuda_stream)
    assert st == 0, S.lib().sl_last_error()
    stream.synchronize()
    return spins.cpu().numpy().reshape(sp.shape), recs.cpu().numpy().reshape(n + 1, 5)


def _lattice(sp, n):
    lat = S.Lattice(sp)
    lat.sweep(n)
    recs = S.records_to_array(lat.measure())
    spins = lat.spins()
    lat.close()
    return spins, recs


CASES = [  # (parameters, sweeps): each call after the first is on a smaller lattice
    (dict(dim=3, L=64, two_s=2, T=3.19, seed=3), 300),
    (dict(L=1024, T=2.269, seed=4), 700),
    (dict(model=S.NORTH_EAST, L=256, c=0.2, seed=5), 520),
    (dict(L=64, T=2.269, init=S.INIT_COLD, seed=1), 1000),
    (dict(model=S.NE_SUBLATTICE, L=64, c=0.3, seed=6, ne_side=16, ne_lambda=8), 40),
    (dict(model=S.NE_COUPLED, L=32, J=1.0, h=0.1, T=2.2, c=0.5, seed=7), 0),
]


def test_static_equals_lattice_entry_points():
    for kw, n in CASES:
        sp = S.Params(record_capacity=n + 1, **kw)
        print(f"case sweep_static {kw} n={n}", flush=True)
        g_s, g_r = _static(sp, n)
        l_s, l_r = _lattice(sp, n)
        np.testing.assert_array_equal(g_r, l_r)
        np.testing.assert_array_equal(g_s, l_s)


def test_static_from_buffer_and_t0():
    from workloads import random_lattice

    sp = S.Params(L=128, two_s=2, T=1.7, seed=9, init=S.INIT_BUFFER, t0=2 ** 32 - 300,
                  record_capacity=301)
    start = torch.from_numpy(random_lattice(sp.shape, two_s=2, seed=2)).cuda()
    cp = sp.c_struct(start.data_ptr())
    spins = torch.empty(sp.nsites, dtype=torch.int8, device="cuda")
    recs = torch.empty(301 * 5, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    assert S.lib().sl_sweep_static(ctypes.byref(cp), 300, spins.data_ptr(), recs.data_ptr(),
                                   stream.cuda_stream) == 0
    stream.synchronize()
    lat = S.Lattice(sp, init_spins=start)
    lat.sweep(300)
    np.testing.assert_array_equal(recs.cpu().numpy().reshape(301, 5), S.records_to_array(lat.measure()))
    np.testing.assert_array_equal(spins.cpu().numpy().reshape(sp.shape), lat.spins())
    lat.close()
    assert S.lib().sl_sweep_static(ctypes.byref(cp), 301, spins.data_ptr(), recs.data_ptr(),
                                   stream.cuda_stream) == 6


def test_static_refuses_large_lattices():
    spins = torch.empty(1, dtype=torch.int8, device="cuda")
    for kw in (dict(L=8192), dict(dim=3, L=512)):
        cp = S.Params(**kw).c_struct()
        st = S.lib().sl_sweep_static(ctypes.byref(cp), 1, spins.data_ptr(), spins.data_ptr(),
                                     torch.cuda.current_stream().cuda_stream)
        assert st == 2, S.lib().sl_last_error()
        assert b"working memory" in S.lib().sl_last_error()
