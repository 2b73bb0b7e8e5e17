"""Continuous-batching job server for lattice simulations.

Requests (lattice parameters plus a sweep count) arrive over time.  The
server keeps every admitted lattice resident in one device arena
(``Batch``), admits queued requests whenever the arena has room for their
footprint and a job slot is free, and advances all resident jobs together in
chunks of sweeps: requests that arrive while others run join the next chunk,
and finished jobs free their space at once.  Each job's records are the ones
the same lattice would produce alone (the batched kernels are schedule
independent).

Latency of a job = completion time - arrival time (queueing included).
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from .spinlat import Batch, Lattice, Params, records_to_array


@dataclass
class Request:
    id: int
    arrival: float      # seconds after the start of the run
    params: Params
    sweeps: int


@dataclass
class Outcome:
    records: np.ndarray  # (sweeps + 1, 5): r_0 .. r_sweeps
    arrival: float
    admitted: float
    finished: float

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def summarize(outcomes, start: float, end: float):
    lat = np.array([o.latency for o in outcomes.values()])
    attempts = sum(int(o.records.shape[0] - 1) for o in outcomes.values())
    return {
        "jobs": len(outcomes),
        "makespan_s": end - start,
        "jobs_per_s": len(outcomes) / (end - start),
        "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
        "sweeps": attempts,
    }


class Server:
    """Admit by footprint, sweep resident jobs in chunks, retire as they finish."""

    def __init__(self, arena_bytes: int, max_jobs: int = 1024, chunk: int = 64,
                 tile_rows: int = 0, device="cuda", flags: int = 0):
        self.chunk = chunk
        self.batch = Batch(arena_bytes, max_jobs=max_jobs, record_capacity=chunk + 1,
                           tile_rows=tile_rows, device=device, flags=flags)

    def run(self, requests, realtime: bool = True):
        """Serve `requests` (sorted by arrival).  With realtime=False every
        request counts as arrived at time 0 (a closed batch).

        Each round drains the records of everything enqueued so far (the one
        synchronisation), frees the jobs whose last sweeps ran in the previous
        chunk, admits what fits, enqueues the next chunk, and only then does
        the host bookkeeping, so that it overlaps the GPU's work."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        b = self.batch
        queue = deque()
        active = {}      # job id -> request, until its outcome is complete
        parts = {}       # request id -> list of record arrays
        admitted = {}
        outcomes = {}
        retiring = []    # jobs given all their sweeps: complete at the next drain
        nxt = 0
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        while len(outcomes) < len(reqs):
            got = b.drain()
            done_at = now()
            # requests of the drained records, before a freed slot is reused
            owner = {jid: active[jid] for jid in got}
            finishing = [active.pop(jid) for jid in retiring]
            for jid in retiring:
                b.remove(jid)  # the stream is idle after the drain
            t = now()
            while nxt < len(reqs) and (not realtime or reqs[nxt].arrival <= t):
                queue.append(reqs[nxt])
                nxt += 1
            while queue:
                r = queue[0]
                jid = b.add(r.params, r.sweeps)
                if jid is None:
                    break  # no room until a job retires
                queue.popleft()
                active[jid] = r
                parts[r.id] = []
                admitted[r.id] = now()
            working = list(active)
            if working:
                b.sweep(self.chunk)
            # host bookkeeping while the chunk runs
            for jid, recs in got.items():
                parts[owner[jid].id].append(recs)
            for r in finishing:
                outcomes[r.id] = Outcome(np.vstack(parts.pop(r.id)), r.arrival, admitted[r.id], done_at)
            retiring = [jid for jid in working if b.status(jid)[1] == 0]
            if not working and len(outcomes) < len(reqs):
                if queue:
                    raise RuntimeError("request does not fit an empty arena")
                if nxt >= len(reqs):
                    raise RuntimeError("server has requests left but nothing to run")
                time.sleep(max(0.0, reqs[nxt].arrival - now()))
        return outcomes, summarize(outcomes, 0.0, now())

    def close(self):
        self.batch.close()


def run_one_per_launch(requests, realtime: bool = True, device="cuda"):
    """Baseline: serve the same requests one at a time, each as its own
    lattice with its own launches, in arrival order."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    outcomes = {}
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    for r in reqs:
        if realtime and r.arrival > now():
            time.sleep(r.arrival - now())
        start = now()
        p = Params(**{**r.params.__dict__, "record_capacity": r.sweeps + 1})
        lat = Lattice(p, device=device)
        lat.sweep(r.sweeps)
        recs = records_to_array(lat.measure())
        lat.close()
        outcomes[r.id] = Outcome(recs, r.arrival, start, now())
    return outcomes, summarize(outcomes, 0.0, now())


def requests_from_workload(items):
    """Requests from workloads.served_requests dicts."""
    out = []
    for it in items:
        p = Params(model=0, dim=it["dim"], L=it["L"], two_s=it["two_s"], T=it["T"],
                   seed=it["seed"], init=1)
        out.append(Request(it["id"], it["arrival"], p, it["sweeps"]))
    return out
