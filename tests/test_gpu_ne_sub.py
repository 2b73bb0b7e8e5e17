"""GPU parity of the North-East model by random sub-lattices (paper Sec. 3.2):
lattice and every record equal to the oracle's, bit for bit, across
sub-lattice sides, lambda, a single sub-lattice (B = L), partial workgroups,
densities with down-flip thresholds below one, resumed runs, buffer starts and
persistence resets; at the benchmarked size too."""
import numpy as np
import pytest

import oracle as O
import paper_1209_0296_amd as S
from helpers import oracle_params, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


def _p(**kw):
    base = dict(model=S.NE_SUBLATTICE, L=64, c=0.3, seed=3, ne_side=32, ne_lambda=16)
    base.update(kw)
    return S.Params(**base)


CASES = [
    dict(),                                            # the paper's B = 32, lambda = 16
    dict(L=128, ne_side=16, ne_lambda=8, c=0.1),
    dict(L=32, ne_side=32, ne_lambda=16, c=0.42),      # one sub-lattice: periodic wrap inside it
    dict(L=64, ne_side=8, ne_lambda=2, c=0.5),         # c = 1/2: every allowed move accepted
    dict(L=64, ne_side=8, ne_lambda=32, c=0.45),       # lambda = P/2: one iteration per launch
    dict(L=128, ne_side=64, ne_lambda=128, c=0.3),     # 64 lanes on one sub-lattice
    dict(L=96, ne_side=32, ne_lambda=4, c=0.25),       # 9 sub-lattices: a partial workgroup
    dict(L=64, ne_side=16, ne_lambda=64, c=0.7),       # up-flips always, down-flips thresholded
    dict(L=256, ne_side=64, ne_lambda=16, c=0.2, seed=2 ** 40 + 7),
    dict(L=64, ne_side=8, ne_lambda=16, c=0.35),
]


@pytest.mark.parametrize("kw", CASES, ids=[str(i) for i in range(len(CASES))])
def test_sub_lattice_sweeps_match_oracle(kw):
    p = _p(**kw)
    n = 9
    g_s, g_r = run_gpu(p, n, chunks=[4, 5])
    o_s, o_r = run_oracle(p, n)
    np.testing.assert_array_equal(g_r, o_r)
    np.testing.assert_array_equal(g_s, o_s)
    assert g_r[1:, 3].sum() > 0  # something moved


def test_resume_and_buffer_start():
    """A run split at sweep 6 and restarted from the copied lattice (t0 = 6)
    equals the unbroken run: the launch index, not the call, picks the words."""
    import torch

    p = _p(L=128, ne_side=16, ne_lambda=8, c=0.35, seed=91)
    o_s, o_r = run_oracle(p, 11)
    a_s, a_r = run_gpu(p, 6)
    q = _p(L=128, ne_side=16, ne_lambda=8, c=0.35, seed=91, t0=6, init=S.INIT_BUFFER)
    b_s, b_r = run_gpu(q, 5, init_spins=a_s)
    np.testing.assert_array_equal(np.vstack([a_r, b_r[1:]]), o_r)
    np.testing.assert_array_equal(b_s, o_s)
    del torch


def test_persistence_reset():
    p = _p(L=64, c=0.2, seed=17)
    lat = S.Lattice(p)
    lat.measure()
    lat.sweep(3)
    lat.measure()
    lat.reset_persistence()
    lat.sweep(4)
    g = S.records_to_array(lat.measure())
    s = lat.spins()
    lat.close()
    op = oracle_params(p)
    o = O.init_lattice(op)
    O.run(op, o, 0, 3)
    O.reset_persistence(op, o)
    r = O.run(op, o, 3, 4)
    np.testing.assert_array_equal(g, r)
    np.testing.assert_array_equal(s, o)


def test_only_the_auto_schedule():
    lat = S.Lattice(_p())
    with pytest.raises(S.SpinlatError):
        lat.set_launch(S.MODE_FUSED, 8, 4)
    lat.set_launch(S.MODE_AUTO)
    lat.close()


def test_benchmarked_size_matches_oracle():
    """L = 4096, B = 32, lambda = 16, c = 0.1 (the NE benchmark): full lattice
    and records after 3 sweeps."""
    p = _p(L=4096, c=0.1, seed=2026, record_capacity=8)
    g_s, g_r = run_gpu(p, 3)
    o_s, o_r = run_oracle(p, 3)
    np.testing.assert_array_equal(g_r, o_r)
    np.testing.assert_array_equal(g_s, o_s)


BAL_CASES = [
    dict(),                                            # B = 32, lambda = 16: 8 iterations per launch
    dict(L=128, ne_side=16, ne_lambda=8, c=0.1),
    dict(L=32, ne_side=32, ne_lambda=16, c=0.42),      # one sub-lattice: periodic wrap inside it
    dict(L=64, ne_side=8, ne_lambda=8, c=0.5),         # lambda = P/8: one iteration per launch
    dict(L=64, ne_side=8, ne_lambda=2, c=0.45),
    dict(L=128, ne_side=64, ne_lambda=128, c=0.3),     # 64 lanes on one sub-lattice
    dict(L=96, ne_side=32, ne_lambda=4, c=0.7),        # partial workgroup, down-flips thresholded
    dict(L=256, ne_side=64, ne_lambda=16, c=0.2, seed=2 ** 40 + 9),
]


@pytest.mark.parametrize("kw", BAL_CASES, ids=[str(i) for i in range(len(BAL_CASES))])
def test_balanced_sweeps_match_oracle(kw):
    kw = dict(kw)
    kw["model"] = S.NE_SUBLATTICE_BALANCED
    p = _p(**kw)
    g_s, g_r = run_gpu(p, 7, chunks=[3, 4])
    o_s, o_r = run_oracle(p, 7)
    np.testing.assert_array_equal(g_r, o_r)
    np.testing.assert_array_equal(g_s, o_s)
    assert g_r[1:, 3].sum() > 0


def test_balanced_benchmark_size_matches_oracle():
    p = _p(model=S.NE_SUBLATTICE_BALANCED, L=4096, c=0.1, seed=2027, record_capacity=8)
    g_s, g_r = run_gpu(p, 2)
    o_s, o_r = run_oracle(p, 2)
    np.testing.assert_array_equal(g_r, o_r)
    np.testing.assert_array_equal(g_s, o_s)
