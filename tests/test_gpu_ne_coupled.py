"""GPU parity of the North-East model with the Ising coupling (Sec. 3.2, J != 0):
the direct, resident and whole-row kernels must reproduce the oracle's lattice
and every record bit for bit, the window schedules (and the row schedules for
a table with a zero threshold) must be refused, and at J = 0, h = -1 and the
T of c the model must equal the J = 0 NE model on the GPU too."""
import math

import numpy as np
import pytest

import paper_1209_0296_amd as S
from helpers import assert_refused, expected_supported, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

SIMPLE = (S.MODE_SIMPLE, 0, 0)
RESIDENT = (S.MODE_RESIDENT, 0, 0)
AUTO = (S.MODE_AUTO, 0, 0)
# whole-row kernels: (mode, rows per strip, words per lane)
ROW = [(S.MODE_FUSED, 0, 0), (S.MODE_HALF, 0, 0), (S.MODE_FUSED, 3, 1), (S.MODE_FUSED, 8, 2),
       (S.MODE_HALF, 5, 4), (S.MODE_FUSED, 4, 2), (S.MODE_HALF_ROWS, 0, 0), (S.MODE_HALF_ROWS, 0, 1)]

RATES = [dict(J=1.0, h=0.0, T=2.269, c=0.5), dict(J=1.0, h=0.3, T=2.0, c=0.6),
         dict(J=-0.7, h=0.2, T=1.5, c=0.4), dict(J=0.5, h=-1.1, T=math.inf, c=0.3)]


def _check(sp, nsweeps, launch=None, chunks=None):
    print(f"case coupled L={sp.L} J={sp.J} h={sp.h} T={sp.T} c={sp.c} n={nsweeps} "
          f"launch={launch} chunks={chunks}", flush=True)
    if launch is not None and not expected_supported(sp, launch):
        assert_refused(sp, launch)
        return None
    g_s, g_r = run_gpu(sp, nsweeps, launch=launch, chunks=chunks)
    o_s, o_r = run_oracle(sp, nsweeps)
    np.testing.assert_array_equal(g_r, o_r)
    np.testing.assert_array_equal(g_s, o_s)
    return g_r


@pytest.mark.parametrize("L", [8, 16, 64, 136, 216, 512, 1024, 1040, 2048])
@pytest.mark.parametrize("rates", range(len(RATES)))
@pytest.mark.parametrize("launch", [SIMPLE, RESIDENT, AUTO] + ROW)
def test_coupled_shapes(L, rates, launch):
    n = 12 if L >= 512 else 30
    sp = S.Params(model=S.NE_COUPLED, L=L, seed=3 + L, record_capacity=64, **RATES[rates])
    _check(sp, n, launch=launch)


def test_coupled_long_run_and_chunks():
    sp = S.Params(model=S.NE_COUPLED, L=64, J=1.0, h=0.05, T=2.4, c=0.55, seed=21,
                  record_capacity=1001)
    _check(sp, 1000)
    _check(sp, 300, launch=SIMPLE, chunks=[1, 7, 100, 192])


def test_coupled_resident_across_launch_chunks():
    """More sweeps than one resident launch runs (4096)."""
    sp = S.Params(model=S.NE_COUPLED, L=32, J=1.0, h=0.1, T=2.2, c=0.6, seed=5,
                  record_capacity=4200)
    _check(sp, 4100, launch=RESIDENT)


@pytest.mark.parametrize("mode", [S.MODE_HALF_WINDOW, S.MODE_FUSED_WINDOW])
def test_window_schedules_refused(mode):
    lat = S.Lattice(S.Params(model=S.NE_COUPLED, L=1024, J=1.0, T=2.5, c=0.5))
    assert lat.get_launch()[0] == S.MODE_FUSED
    with pytest.raises(S.SpinlatError) as e:
        lat.set_launch(mode, 0, 0)
    assert e.value.status == 2
    lat.close()


def test_zero_thresholds_use_the_direct_kernel():
    """T -> 0+: thresholds of energy-raising moves are 0, which the row
    kernels' 32-bit "word <= thr - 1" cannot hold; AUTO takes the direct
    kernel, the row schedules are refused, and the result is the oracle's."""
    sp = S.Params(model=S.NE_COUPLED, L=1024, J=1.0, h=0.1, T=1e-300, c=0.6, seed=4,
                  record_capacity=16)
    lat = S.Lattice(sp)
    assert lat.get_launch()[0] == S.MODE_SIMPLE
    for mode in (S.MODE_HALF, S.MODE_FUSED):
        with pytest.raises(S.SpinlatError) as e:
            lat.set_launch(mode, 0, 0)
        assert e.value.status == 2
    lat.close()
    _check(sp, 6)


def test_zero_coupling_equals_the_ne_model_on_the_gpu():
    c = 0.3
    T = 2.0 / math.log((1.0 - c) / c)
    a = S.Params(model=S.NE_COUPLED, L=256, J=0.0, h=-1.0, T=T, c=c, seed=9, record_capacity=64)
    b = S.Params(model=S.NORTH_EAST, L=256, c=c, seed=9, record_capacity=64)
    for launch in (SIMPLE, AUTO):
        ga, ra = run_gpu(a, 40, launch=launch)
        gb, rb = run_gpu(b, 40, launch=launch)
        np.testing.assert_array_equal(ga, gb)
        np.testing.assert_array_equal(ra, rb)


def test_coupled_persistence_reset():
    import oracle as O
    from helpers import oracle_params

    sp = S.Params(model=S.NE_COUPLED, L=64, J=1.0, h=0.2, T=2.0, c=0.6, seed=13, record_capacity=64)
    lat = S.Lattice(sp)
    lat.sweep(10)
    lat.measure()
    lat.reset_persistence()
    lat.sweep(5)
    r2 = S.records_to_array(lat.measure())
    spins = lat.spins()
    lat.close()
    op = oracle_params(sp)
    s = O.init_lattice(op)
    O.run(op, s, 0, 10, records=False)
    O.reset_persistence(op, s)
    rec = O.run(op, s, 10, 5)
    np.testing.assert_array_equal(r2, rec)
    np.testing.assert_array_equal(spins, s)
