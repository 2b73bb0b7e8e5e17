"""GPU parity of sl_overlap (the overlap with a reference lattice behind Phi(t)
of Eq. 4) and of a Phi(t) series, against the oracle's observables."""
import numpy as np
import pytest

import oracle as O
from oracle import observables as OB
import paper_1209_0296_amd as S
from helpers import oracle_params

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kw", [
    dict(L=64, T=2.269),
    dict(dim=3, L=24, two_s=2, T=3.0),
    dict(model=S.NORTH_EAST, L=128, c=0.3),
    dict(model=S.NE_SUBLATTICE, L=128, c=0.45, ne_side=16, ne_lambda=8),
])
def test_overlap_series_matches_oracle(kw):
    p = S.Params(seed=77, **kw)
    op = oracle_params(p)
    lat = S.Lattice(p)
    ref = lat.copy_spins()
    o = O.init_lattice(op)
    o_ref = o.copy()
    np.testing.assert_array_equal(ref.cpu().numpy(), o_ref)
    t = 0
    for step in (0, 3, 7, 20):
        if step:
            lat.sweep(step)
            lat.measure()
            O.run(op, o, t, step)
            t += step
        got = lat.overlap(ref)
        want = OB.overlap(op, o, o_ref)
        assert got == want, (t, got, want)
        if p.model != S.ISING:
            assert S.autocorrelation(p, got) == pytest.approx(OB.autocorrelation(op, want), rel=1e-15)
    lat.close()


def test_overlap_with_itself_and_with_a_buffer():
    import torch

    p = S.Params(L=96, T=2.0, seed=5)
    lat = S.Lattice(p)
    me = lat.copy_spins()
    assert lat.overlap(me) == 96 * 96
    flipped = (-me).contiguous()
    assert lat.overlap(flipped) == -96 * 96
    rng = np.random.default_rng(1)
    other = (2 * rng.integers(0, 2, size=(96, 96)) - 1).astype(np.int8)
    want = int(np.sum(me.cpu().numpy().astype(np.int64) * other))
    assert lat.overlap(torch.from_numpy(other)) == want
    lat.close()
