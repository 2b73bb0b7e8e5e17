"""The autotuner picks a schedule that fits, is at least as fast as the
default on its own probe, and leaves results unchanged."""
import numpy as np
import pytest

import paper_1209_0296_amd as S
from paper_1209_0296_amd.autotune import autotune, candidates
from helpers import run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kw", [dict(L=256, T=2.269), dict(dim=3, L=48, two_s=2, T=3.2),
                                dict(model=S.NORTH_EAST, L=512, c=0.2),
                                dict(model=S.NE_COUPLED, L=512, J=1.0, h=0.1, T=2.2, c=0.6)])
def test_autotuned_schedule_runs_and_matches(kw):
    p = S.Params(seed=3, record_capacity=32, **kw)
    best, table = autotune(p, sweeps=20, warmup=10)
    assert best in table and len(table) >= 3
    assert table[best] == min(table.values())
    assert all(c in candidates(p) for c in table)
    if p.model == S.NE_COUPLED:  # the window schedules refuse coupled lattices
        assert all(c[0] not in (S.MODE_HALF_WINDOW, S.MODE_FUSED_WINDOW) for c in table)
    g_s, g_r = run_gpu(p, 9, launch=best)
    o_s, o_r = run_oracle(p, 9)
    np.testing.assert_array_equal(g_r, o_r)
    np.testing.assert_array_equal(g_s, o_s)
