"""The oracle still reproduces its frozen output for the L=32 square-lattice
workload (tests/golden/c1_oracle.txt, written by tests/golden/make_golden.py)."""
import hashlib
import os

import numpy as np

import oracle
from paper_1110_0899_amd import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


def read_golden():
    vals, recs = {}, []
    with open(os.path.join(HERE, "golden", "c1_oracle.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if len(parts) == 2:
                vals[parts[0]] = parts[1]
            else:
                recs.append([int(v) for v in parts])
    return vals, np.array(recs, dtype=np.int64)


def test_oracle_matches_golden():
    vals, recs = read_golden()
    c = workloads.C1
    thr = oracle.threshold(1.0, c["T"])
    assert thr == int(vals["threshold"])
    S = oracle.init_spins(c["dim"], c["L"], c["seed"])
    assert hashlib.sha256(S.tobytes()).hexdigest() == vals["init_spins_sha256"]
    rec = oracle.run(c["dim"], c["L"], thr, c["seed"], 0, c["n_meas"], S)
    assert hashlib.sha256(S.tobytes()).hexdigest() == vals["final_spins_sha256"]
    assert int(rec[:, 2].sum()) == int(vals["sum_csize"])
    assert int(rec[:, 0].sum()) == int(vals["sum_B"])
    assert int(rec[:, 1].sum()) == int(vals["sum_M"])
    assert (rec[: len(recs), :] == recs[:, 1:]).all()
