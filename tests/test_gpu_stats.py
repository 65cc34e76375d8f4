"""The counting build (libwolff_stats.so, the library compiled with
WOLFF_STATS=1): its records and spins equal the CPU oracle's (counting must
not change the method), and its counters agree with what the records fix:
the sites expanded are the sum of |C| over the updates, the updates are
the number run, every path issues global reads and writes, and only the
team path claims with global atomics.  Runs in a child process, which
loads the counting build in place of libwolff.so."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import json, numpy as np
import oracle
from paper_1110_0899_amd import binding, workloads
binding.load()
assert binding.LIBRARY.endswith("libwolff_stats.so")
out = []
for dim, L, T, path, slab in [(2, 64, workloads.TC_2D, binding.PATH_LDS, 0),
                              (2, 64, workloads.TC_2D, binding.PATH_LDS, 1024),
                              (2, 64, workloads.TC_2D, binding.PATH_SINGLE, 0),
                              (2, 64, workloads.TC_2D, binding.PATH_TEAM, 0),
                              (3, 16, workloads.T_3D, binding.PATH_LDS, 0),
                              (3, 16, workloads.T_3D, binding.PATH_TEAM, 0),
                              (2, 37, 2.4, binding.PATH_SINGLE, 0)]:
    n, seed = 150, 5
    with binding.Simulation(dim, L, 1.0, T, seed) as sim:
        if slab:
            sim.set_lds_slab(slab)
        sim.set_path(path)
        sim.stats(reset=True)
        sim.run(n)
        rec = sim.observables()
        c = sim.stats()
        S = sim.spins()
    S0 = oracle.init_spins(dim, L, seed)
    ref = oracle.run(dim, L, oracle.threshold(1.0, T), seed, 0, n, S0)
    got = np.stack([rec["bond_sum"], rec["mag"], rec["csize"]], axis=1)
    out.append({"case": [dim, L, T, path, slab], "match": bool((got == ref).all() and (S == S0).all()),
                "sum_csize": int(ref[:, 2].sum()), "n": n, "counters": c})
jobs = [workloads.Job(2, 32, workloads.TC_2D, 7, 60), workloads.Job(3, 8, workloads.T_3D, 8, 60),
        workloads.Job(2, 48, 2.2, 9, 60)]
for lds in (True, False):
    with binding.Batch(jobs) as b:
        b.set_lds(lds)
        b.stats(reset=True)
        b.run()
        recs = [b.records(i) for i in range(len(jobs))]
        c = b.stats()
    out.append({"case": ["batch", lds], "sum_csize": int(sum(int(r["csize"].sum()) for r in recs)),
                "n": 3 * 60, "counters": c, "match": True})
print(json.dumps(out))
'''


def test_counting_build_matches_oracle_and_counts():
    env = dict(os.environ, WOLFF_LIBRARY="stats")
    assert os.path.exists(os.path.join(ROOT, "paper_1110_0899_amd", "libwolff_stats.so"))
    p = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=240)
    assert p.returncode == 0, p.stderr[-3000:]
    results = json.loads(p.stdout.strip().splitlines()[-1])
    for r in results:
        c = r["counters"]
        print(r["case"], {k: c[k] for k in ("sites", "steps", "read_bytes", "write_bytes",
                                            "atomic_bytes", "messages")}, flush=True)
        assert r["match"], r["case"]
        assert c["sites"] == r["sum_csize"], r["case"]
        assert c["updates"] == r["n"], r["case"]
        assert c["steps"] > 0 and c["read_bytes"] > 0 and c["write_bytes"] > 0, r["case"]
        assert c["claims"] >= c["sites"] - r["n"], r["case"]    # every member but the seed was claimed
        path = r["case"][3] if r["case"][0] != "batch" else None
        if path == 2:                                            # the team path claims with atomics
            assert c["atomic_bytes"] >= 4 * (c["sites"] - r["n"])
        if path == 3 and r["case"][4]:                           # LDS path on several slabs
            assert c["messages"] > 0
