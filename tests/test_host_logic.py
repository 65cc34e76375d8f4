"""Host-side logic that needs no GPU: the seeded workload generators, the
autotuner's cache, the serving statistics and the Potts critical
temperature used by the benchmarks."""
import json
import math
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1110_0899_amd import autotune, serve, workloads


def test_c4_replica_set():
    jobs = workloads.c4_jobs(7)
    assert len(jobs) == 320
    two, three = jobs[:256], jobs[256:]
    assert all(j.dim == 2 and j.L in (64, 128, 256, 512, 1024) and 2.0 <= j.T <= 2.6 for j in two)
    assert all(j.dim == 3 and j.L in (32, 64, 128) and 4.3 <= j.T <= 4.7 for j in three)
    assert [j.seed for j in jobs] == [0x40000000 + r for r in range(320)]
    assert all(j.n_updates == 7 and j.q == 0 for j in jobs)
    assert workloads.c4_jobs(7) == jobs                      # seeded: the list is the contract


def test_c5_stream():
    jobs = workloads.c5_stream(n_jobs=400, rate_per_s=50.0, seed=5)
    assert len(jobs) == 400
    t = np.array([j.arrival_s for j in jobs])
    assert (np.diff(t) > 0).all()
    # Poisson arrivals: mean gap 1/rate within a few standard errors
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 1 / 50.0) < 4 * (1 / 50.0) / math.sqrt(400)
    for j in jobs:
        tc = workloads.TC_2D if j.dim == 2 else workloads.T_3D
        lo, hi = (64, 4096) if j.dim == 2 else (32, 256)
        assert lo <= j.L <= hi
        assert abs(j.T / tc - 1.0) <= 0.02 + 1e-12
        assert 100 <= j.n_updates <= 10000
    assert 0.35 < np.mean([j.dim == 2 for j in jobs]) < 0.65
    assert [j.seed for j in jobs] == [0x50000000 + k for k in range(400)]


def test_same_shape_jobs_and_potts_tc():
    jobs = workloads.same_shape_jobs(3, 16, 5, 9)
    assert {(j.dim, j.L, j.T, j.n_updates, j.q) for j in jobs} == {(3, 16, workloads.T_3D, 9, 0)}
    p = workloads.same_shape_jobs(2, 8, 2, 4, q=3)
    assert all(j.q == 3 and j.T == workloads.potts_tc_2d(3) for j in p)
    # q = 2 Potts at coupling J is Ising at J/2: T_c halves
    assert workloads.potts_tc_2d(2) == pytest.approx(workloads.TC_2D / 2, rel=1e-14)
    # self-dual point of the q = 3 and q = 4 models
    assert workloads.potts_tc_2d(3) == pytest.approx(0.99497, abs=1e-5)
    assert workloads.potts_tc_2d(4) == pytest.approx(1.0 / math.log(3.0), rel=1e-14)


def test_tuner_keys_and_cache(tmp_path, monkeypatch):
    monkeypatch.setenv("WOLFF_TUNE_CACHE", str(tmp_path / "tune.json"))
    k = autotune.key(2, 4096, 2048)
    assert k.endswith("|d2|L2^12|B2^11")
    assert autotune.key(2, 4096, 2048, q=3) == k + "|potts"
    assert autotune.key(3, 200, 1000) == autotune.key(3, 256, 1024)   # classes by powers of two
    # a cached entry is returned without measuring anything
    jobs = workloads.same_shape_jobs(2, 4096, 2048, 16)
    entry = {"wg": 512, "queue_entries": 2048, "key": k}
    (tmp_path / "tune.json").write_text(json.dumps({k: entry}))
    assert autotune.tune(jobs) == entry
    autotune._store("other", {"wg": 64})
    cached = json.loads((tmp_path / "tune.json").read_text())
    assert cached[k] == entry and cached["other"] == {"wg": 64}
    assert all(wg <= 1024 and q >= wg and q & (q - 1) == 0 for wg, q in autotune.CANDIDATES)


def test_tuner_key_of_mixed_sets():
    # a same-class set keys by its class; a mixed set (C4) never shares that
    # key, and its key follows the multiset of shapes, not the job order
    same = workloads.same_shape_jobs(2, 512, 320, 8)
    assert autotune.set_key(same) == autotune.key(2, 512, 320)
    mixed = workloads.c4_jobs(8)
    k = autotune.set_key(mixed)
    assert k.startswith(autotune.key(3, 128, len(mixed)) + "|mixed:")   # largest shape: 3D L=128
    assert autotune.set_key(list(reversed(mixed))) == k
    assert autotune.set_key(mixed[:-1]) != k
    # classes round L up to powers of two: L = 200 and 256 share one
    a = [workloads.Job(3, 200, 4.5, 1, 8), workloads.Job(3, 256, 4.5, 2, 8)]
    assert autotune.set_key(a) == autotune.key(3, 256, 2)


def test_serving_percentiles():
    xs = list(range(1, 101))
    assert serve.percentile(xs, 50) == pytest.approx(50.5)
    assert serve.percentile(xs, 99) == pytest.approx(99.01)
    assert math.isnan(serve.percentile([], 50))


def test_bench_refuses_several_gpus():
    # one GPU only: --gpus above 1 exits with a message before touching a device
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=root, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_stat_names_follow_the_header():
    # the binding names the counting build's counters in the header's order
    import re
    from paper_1110_0899_amd import binding
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    text = open(os.path.join(root, "include", "wolff.h")).read()
    defs = {m.group(1): int(m.group(2))
            for m in re.finditer(r"#define WOLFF_STAT_([A-Z_]+)\s+(\d+)", text)}
    count = defs.pop("COUNT")
    assert sorted(defs.values()) == list(range(count))
    assert binding.STAT_COUNT == count == len(binding.STAT_NAMES)
    for name, idx in defs.items():
        assert binding.STAT_NAMES[idx] == name.lower(), (name, idx)
