"""The server's scheduling on the CPU: admission, chunked sweeps, draining and
retirement, with job slots reused as soon as they free.  A stand-in batch with
the library batch's record semantics (r_0 at admission, one record per sweep,
a ring of record_capacity records, a job table of max_jobs slots given out
lowest first) tags every record with its request, so a record delivered to the
wrong request, lost or duplicated fails the check."""
import numpy as np
import pytest

from paper_1209_0296_amd.serve import Request, Server


class StandInBatch:
    def __init__(self, max_jobs, record_capacity, arena_jobs):
        self.max_jobs, self.cap, self.arena_jobs = max_jobs, record_capacity, arena_jobs
        self.jobs = {}  # slot -> dict(tag, t, remaining, pending)

    def add(self, params, sweeps):
        if len(self.jobs) >= min(self.max_jobs, self.arena_jobs):
            return None
        jid = next(j for j in range(self.max_jobs) if j not in self.jobs)
        self.jobs[jid] = dict(tag=params.seed, t=0, remaining=sweeps, pending=[0])
        return jid

    def sweep(self, n):
        for job in self.jobs.values():
            budget = min(n, job["remaining"], self.cap - len(job["pending"]))
            for _ in range(budget):
                job["t"] += 1
                job["pending"].append(job["t"])
            job["remaining"] -= budget

    def drain(self):
        out = {}
        for jid, job in self.jobs.items():
            if job["pending"]:
                out[jid] = np.array([[t, job["tag"], 0, 0, 0] for t in job["pending"]], dtype=np.int64)
                job["pending"] = []
        return out

    def status(self, jid):
        job = self.jobs[jid]
        return job["t"], job["remaining"], len(job["pending"])

    def remove(self, jid):
        del self.jobs[jid]


class P:
    def __init__(self, seed):
        self.seed = seed


def _server(max_jobs, chunk, arena_jobs):
    srv = Server.__new__(Server)  # the scheduling logic alone, on a stand-in batch
    srv.chunk = chunk
    srv.batch = StandInBatch(max_jobs, chunk + 1, arena_jobs)
    return srv


@pytest.mark.parametrize("max_jobs,chunk,arena_jobs", [(3, 4, 3), (2, 1, 5), (8, 16, 4), (1, 7, 1)])
def test_every_request_gets_exactly_its_records(max_jobs, chunk, arena_jobs):
    rng = np.random.default_rng(max_jobs * 100 + chunk)
    reqs = [Request(i, 0.0, P(1000 + i), int(rng.integers(0, 40))) for i in range(23)]
    outcomes, stats = _server(max_jobs, chunk, arena_jobs).run(reqs, realtime=False)
    assert stats["jobs"] == len(reqs) and set(outcomes) == {r.id for r in reqs}
    for r in reqs:
        rec = outcomes[r.id].records
        np.testing.assert_array_equal(rec[:, 0], np.arange(r.sweeps + 1))  # r_0 .. r_sweeps, in order
        assert (rec[:, 1] == r.params.seed).all()                         # all of them its own
        assert outcomes[r.id].finished >= outcomes[r.id].admitted


def test_realtime_arrivals_wait_and_finish():
    reqs = [Request(i, 0.002 * i, P(50 + i), 5 + i) for i in range(6)]
    outcomes, _ = _server(2, 3, 2).run(reqs, realtime=True)
    for r in reqs:
        np.testing.assert_array_equal(outcomes[r.id].records[:, 0], np.arange(r.sweeps + 1))
        assert outcomes[r.id].admitted >= r.arrival


def test_request_too_big_for_an_empty_arena_raises():
    with pytest.raises(RuntimeError):
        _server(2, 3, 0).run([Request(0, 0.0, P(1), 3)], realtime=False)
