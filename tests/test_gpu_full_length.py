"""The benchmarked configurations at their stated length, in the schedule the
benchmark times: the GPU lattice and record series must hash to the oracle's
golden values (tests/golden/*.json, written by tests/golden/make_golden.py from
the oracle alone) at every checkpoint the golden file holds."""
import glob
import hashlib
import json
import os

import numpy as np
import pytest

import paper_1209_0296_amd as S

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FILES = sorted(glob.glob(os.path.join(GOLDEN, "*.json")))
MODELS = {"ising": S.ISING, "north_east": S.NORTH_EAST}


def _params(doc, capacity):
    q = doc["params"]
    return S.Params(model=MODELS[q["model"]], dim=q["dim"], L=q["L"], two_s=q["two_s"], J=q["J"],
                    h=q["h"], T=q["T"], c=q["c"], seed=q["seed"], t0=q["t0"],
                    init=S.INIT_COLD if q["init"] == "cold" else S.INIT_RANDOM,
                    record_capacity=capacity)


@pytest.mark.parametrize("path", FILES, ids=[os.path.basename(f)[:-5] for f in FILES])
def test_golden_hashes(path):
    doc = json.load(open(path))
    cps = doc["checkpoints"]
    assert cps, "golden file without checkpoints"
    step = cps[0]["sweeps"]
    sp = _params(doc, capacity=step + 1)
    print(f"case golden {doc['case']}: {cps[-1]['sweeps']} of {doc['sweeps']} sweeps", flush=True)
    lat = S.Lattice(sp)  # default (AUTO) schedule, as benchmarked
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(S.records_to_array(lat.measure()), dtype="<i8").tobytes())
    done = 0
    for cp in cps:
        while done < cp["sweeps"]:
            n = min(step, cp["sweeps"] - done)
            lat.sweep(n)
            recs = np.ascontiguousarray(S.records_to_array(lat.measure()), dtype="<i8")
            assert len(recs) == n
            h.update(recs.tobytes())
            done += n
        assert [int(v) for v in recs[-1]] == cp["last_record"], f"record at sweep {done}"
        assert h.copy().hexdigest() == cp["records_sha256"], f"record series at sweep {done}"
        spins = np.ascontiguousarray(lat.spins())
        assert hashlib.sha256(spins.tobytes()).hexdigest() == cp["lattice_sha256"], f"lattice at {done}"
    lat.close()
