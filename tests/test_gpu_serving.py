"""Batched and serving forms: every replica / job gives exactly the records it
gives alone (same seed, same update indices), whatever else shares the
launch, and the serving loop respects its HBM budget."""
import numpy as np
import pytest
import torch

import oracle
from paper_1110_0899_amd import binding, workloads

pytestmark = pytest.mark.gpu

TC2, T3 = workloads.TC_2D, workloads.T_3D


def as_array(rec):
    return np.stack([rec["bond_sum"], rec["mag"], rec["csize"]], axis=1)


def alone(job, start=0):
    with binding.Simulation(job.dim, job.L, job.J, job.T, job.seed) as sim:
        sim.set_path(binding.PATH_SINGLE)
        if start:
            sim.set_spins(np.full(job.L ** job.dim, start, dtype=np.int8), 0)
        sim.run(job.n_updates)
        return as_array(sim.observables()), sim.spins()


def mixed_jobs(n, seed=0):
    rng = np.random.default_rng(seed)
    jobs = []
    for k in range(n):
        if rng.random() < 0.5:
            L = int(rng.choice([4, 7, 16, 31, 64, 100]))
            jobs.append(workloads.Job(2, L, float(TC2 * (1 + rng.uniform(-0.1, 0.1))),
                                      0x50000000 + k, int(rng.integers(20, 300))))
        else:
            L = int(rng.choice([3, 6, 8, 13, 20]))
            jobs.append(workloads.Job(3, L, float(T3 * (1 + rng.uniform(-0.1, 0.1))),
                                      0x50000000 + k, int(rng.integers(20, 300))))
    return jobs


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available()
    binding.load()


def test_batch_budgeted_quanta_match_alone():
    jobs = mixed_jobs(24, seed=1)
    with binding.Batch(jobs) as b:
        for _ in range(200):
            if all(b.progress(i)[0] == 0 for i in range(len(jobs))):
                break
            b.run(7)
        for i, j in enumerate(jobs):
            got = as_array(b.records(i))
            ref, S = alone(j)
            assert (got == ref).all(), i
            assert (b.spins(i) == S).all(), i


def test_mixed_c4_style_batch_against_oracle():
    # small version of the mixed replica set (2D and 3D, spread of L and T)
    rng = np.random.default_rng(4)
    jobs = [workloads.Job(2, int(rng.choice([8, 16, 32])), float(rng.uniform(2.0, 2.6)),
                          0x40000000 + r, 150) for r in range(12)]
    jobs += [workloads.Job(3, int(rng.choice([4, 8])), float(rng.uniform(4.3, 4.7)),
                           0x40000000 + 12 + r, 150) for r in range(6)]
    with binding.Batch(jobs) as b:
        b.run()
        for i, j in enumerate(jobs):
            thr = oracle.threshold(j.J, j.T)
            S = oracle.init_spins(j.dim, j.L, j.seed)
            ref = oracle.run(j.dim, j.L, thr, j.seed, 0, j.n_updates, S)
            assert (as_array(b.records(i)) == ref).all(), i
            assert (b.spins(i) == S).all(), i


def test_server_alone_vs_mix():
    jobs = mixed_jobs(40, seed=2)
    results = {}
    with binding.Server() as srv:
        ids = {}
        # submit in waves between quanta: later jobs join while earlier ones run
        for wave in range(4):
            for k in range(wave * 10, wave * 10 + 10):
                ids[srv.submit(jobs[k])] = k
            srv.step(0.5)
        while len(results) < len(jobs):
            srv.step(0.5)
            for jid in srv.finished():
                results[ids[jid]] = as_array(srv.take(jid))
        st = srv.stats()
    assert st["running"] == 0 and st["queued"] == 0
    for k, j in enumerate(jobs):
        ref, _ = alone(j)
        assert (results[k] == ref).all(), k


def test_server_admission_by_footprint():
    # budget for about two jobs at once: the rest wait in the queue
    jobs = [workloads.Job(2, 64, TC2, 77 + k, 60) for k in range(6)]
    fp = 64 * 64 * 5 + 60 * 24 + 2048
    with binding.Server(hbm_budget_bytes=int(2.2 * fp)) as srv:
        ids = {srv.submit(j): k for k, j in enumerate(jobs)}
        results = {}
        while len(results) < len(jobs):
            srv.step(0.2)
            st = srv.stats()
            assert st["resident_bytes"] <= st["budget_bytes"]
            assert st["running"] <= 2
            for jid in srv.finished():
                results[ids[jid]] = as_array(srv.take(jid))
    for k, j in enumerate(jobs):
        ref, _ = alone(j)
        assert (results[k] == ref).all(), k


def test_server_rejects_oversized_job():
    with binding.Server(hbm_budget_bytes=1 << 16) as srv:
        with pytest.raises(binding.WolffError) as e:
            srv.submit(workloads.Job(2, 1024, TC2, 1, 10))
        assert e.value.code == binding.EINVAL


def test_server_update_only_jobs():
    jobs = mixed_jobs(12, seed=3)
    results = {}
    with binding.Server() as srv:
        ids = {srv.submit(j, update_only=True): k for k, j in enumerate(jobs)}
        while len(results) < len(jobs):
            srv.step(1.0)
            for jid in srv.finished():
                results[ids[jid]] = as_array(srv.take(jid))
    for k, j in enumerate(jobs):
        ref, _ = alone(j)
        assert (results[k][:, 0] == binding.NOT_MEASURED).all()
        assert (results[k][:, 1:] == ref[:, 1:]).all(), k
