"""Continuous batching: requests arriving while others run are admitted as
memory frees up, and every result equals the same lattice run alone."""
import numpy as np
import pytest

import paper_1209_0296_amd as S
from paper_1209_0296_amd.serve import Request, Server, run_one_per_launch
from helpers import run_oracle

pytestmark = pytest.mark.gpu


def _requests():
    rng = np.random.default_rng(3)
    reqs = []
    t = 0.0
    for i in range(24):
        t += rng.exponential(0.01)
        dim = 2 if i % 3 else 3
        L = int(rng.choice([32, 40, 64, 96, 128])) if dim == 2 else int(rng.choice([16, 24, 32]))
        two_s = 1 + (i % 2)
        T = (2.2 if dim == 2 else 4.3) if two_s == 1 else (1.6 if dim == 2 else 3.0)
        p = S.Params(dim=dim, L=L, two_s=two_s, T=T * float(rng.uniform(0.9, 1.1)), seed=500 + i)
        reqs.append(Request(i, t, p, int(rng.integers(20, 70))))
    return reqs


def test_served_results_equal_alone_runs():
    reqs = _requests()
    # room for only a few jobs at a time: later requests wait for retirements
    cfg = S.batch_config(max_jobs=64, record_capacity=17)
    biggest = max(S.batch_job_bytes(r.params, cfg) for r in reqs)
    arena = S.batch_base_bytes(cfg) + 3 * biggest
    srv = Server(arena, max_jobs=64, chunk=16)
    outcomes, stats = srv.run(reqs, realtime=True)
    srv.close()
    assert stats["jobs"] == len(reqs)
    base, _ = run_one_per_launch(reqs, realtime=False)
    for r in reqs:
        o_s, o_r = run_oracle(r.params, r.sweeps)
        np.testing.assert_array_equal(outcomes[r.id].records, o_r)
        np.testing.assert_array_equal(base[r.id].records, o_r)
        assert outcomes[r.id].finished >= outcomes[r.id].admitted >= 0.0
    # admission really was limited by the arena: some job waited in the queue
    waits = [outcomes[r.id].admitted - r.arrival for r in reqs]
    assert max(waits) > 0.0
