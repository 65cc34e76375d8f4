"""q-state Potts on the GPU against the CPU oracle, bit for bit: records
(B, M, |C|) after every update and the final colours, through the C ABI."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1110_0899_amd import binding, workloads

pytestmark = pytest.mark.gpu


def tc_potts_2d(q):
    return 1.0 / math.log(1.0 + math.sqrt(q))


def as_array(rec):
    return np.stack([rec["bond_sum"], rec["mag"], rec["csize"]], axis=1)


def oracle_potts(dim, L, q, J, T, seed, n, C=None):
    thr = oracle.potts_threshold(J, T)
    if C is None:
        C = oracle.potts_init(dim, L, q, seed)
    return oracle.potts_run(dim, L, q, thr, seed, 0, n, C), C


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available()
    binding.load()


CASES = [
    (2, 16, 3, tc_potts_2d(3), 5, 400),
    (2, 32, 4, tc_potts_2d(4), 6, 300),
    (2, 48, 3, 0.8, 7, 120),          # tiled storage, ordered phase
    (2, 17, 5, tc_potts_2d(5), 8, 300),  # odd L
    (2, 2, 3, 0.7, 9, 100),           # L = 2 multigraph
    (3, 8, 3, 1.8, 10, 300),
    (3, 16, 3, 1.7, 11, 80),          # tiled 3D
    (3, 5, 4, 1.5, 12, 200),
    (2, 24, 10, 0.7, 13, 200),
]


@pytest.mark.parametrize("dim,L,q,T,seed,n", CASES)
def test_potts_single_matches_oracle(dim, L, q, T, seed, n):
    print("case potts dim=%d L=%d q=%d T=%.4f seed=%d" % (dim, L, q, T, seed), flush=True)
    ref, Cref = oracle_potts(dim, L, q, 1.0, T, seed, n)
    with binding.Simulation(dim, L, 1.0, T, seed, q=q) as sim:
        assert sim.info().q == q
        assert sim.info().threshold == oracle.potts_threshold(1.0, T)
        sim.run(n // 2)
        sim.run(n - n // 2)
        got = as_array(sim.observables())
        C = sim.spins()
    assert (got == ref).all()
    assert (C == Cref).all()


def test_potts_q2_is_ising():
    # q = 2 at J = 2 is the Ising update at J = 1: same records, colour 0 = +1
    for dim, L, T, seed, n in [(2, 32, workloads.TC_2D, 21, 300), (3, 12, workloads.T_3D, 22, 200)]:
        with binding.Simulation(dim, L, 1.0, T, seed) as a, \
                binding.Simulation(dim, L, 2.0, T, seed, q=2) as b:
            a.set_path(binding.PATH_SINGLE)
            a.run(n)
            b.run(n)
            ra, rb = as_array(a.observables()), as_array(b.observables())
            Sa, Cb = a.spins(), b.spins()
        assert (ra == rb).all()
        assert (Sa == 1 - 2 * Cb.astype(np.int16)).all()


def test_potts_batch_mixed_with_ising():
    jobs = [workloads.Job(2, 32, tc_potts_2d(3), 31, 200, q=3),
            workloads.Job(2, 32, workloads.TC_2D, 32, 200),
            workloads.Job(3, 8, 1.8, 33, 150, q=3),
            workloads.Job(2, 20, tc_potts_2d(4), 34, 150, q=4),
            workloads.Job(3, 6, workloads.T_3D, 35, 150)]
    with binding.Batch(jobs) as b:
        b.run(70)
        b.run()
        for i, j in enumerate(jobs):
            got = as_array(b.records(i))
            if j.q:
                ref, Cref = oracle_potts(j.dim, j.L, j.q, 1.0, j.T, j.seed, j.n_updates)
            else:
                Cref = oracle.init_spins(j.dim, j.L, j.seed)
                ref = oracle.run(j.dim, j.L, oracle.threshold(1.0, j.T), j.seed, 0, j.n_updates, Cref)
            assert (got == ref).all(), i
            assert (b.spins(i) == Cref).all(), i


def test_potts_update_only_and_ordered_start():
    dim, L, q, T, seed, n = 2, 40, 3, 0.9, 41, 150
    C0 = np.zeros(L * L, dtype=np.int8)
    ref, Cref = oracle_potts(dim, L, q, 1.0, T, seed, n, C0.copy())
    with binding.Batch([workloads.Job(dim, L, T, seed, n, q=q)], start=1, update_only=True) as b:
        b.run()
        got = as_array(b.records(0))
        assert (b.spins(0) == Cref).all()
    assert (got[:, 0] == binding.NOT_MEASURED).all()
    assert (got[:, 1:] == ref[:, 1:]).all()


def test_potts_set_spins_and_paths():
    # colours set from the host; the one-workgroup and the team path take
    # turns on the same lattice (each claims with its own mechanism)
    dim, L, q, T, seed = 2, 16, 4, 0.9, 51
    rng = np.random.default_rng(3)
    C = rng.integers(0, q, size=L * L).astype(np.int8)
    ref, Cref = oracle_potts(dim, L, q, 1.0, T, seed, 120, C.copy())
    with binding.Simulation(dim, L, 1.0, T, seed, q=q) as sim:
        with pytest.raises(binding.WolffError):
            sim.set_spins(np.full(L * L, q, dtype=np.int8), 0)
        sim.set_spins(C, 0)
        assert sim.info().path == binding.PATH_SINGLE
        sim.run(40)
        sim.set_path(binding.PATH_TEAM, 8)
        sim.run(40)
        sim.set_path(binding.PATH_SINGLE)
        sim.set_measure(False)
        sim.run(20)
        sim.set_measure(True)
        sim.set_path(binding.PATH_TEAM, 8)
        sim.run(20)
        got = as_array(sim.observables())
        assert (sim.spins() == Cref).all()
    assert (got[:80] == ref[:80]).all()
    assert (got[80:100, 0] == binding.NOT_MEASURED).all() and (got[80:100, 1:] == ref[80:100, 1:]).all()
    assert (got[100:] == ref[100:]).all()


@pytest.mark.parametrize("dim,L,q,T,seed,n", [(2, 64, 3, tc_potts_2d(3), 71, 120),
                                              (2, 33, 4, 0.85, 72, 100),
                                              (3, 16, 3, 1.7, 73, 80),
                                              (2, 1024, 3, tc_potts_2d(3), 74, 6)])
def test_potts_team_path_matches_oracle(dim, L, q, T, seed, n):
    print("case potts team dim=%d L=%d q=%d" % (dim, L, q), flush=True)
    ref, Cref = oracle_potts(dim, L, q, 1.0, T, seed, n)
    with binding.Simulation(dim, L, 1.0, T, seed, q=q) as sim:
        sim.set_path(binding.PATH_TEAM, 16)
        sim.run(n)
        got = as_array(sim.observables())
        C = sim.spins()
    assert (got == ref).all()
    assert (C == Cref).all()


def test_potts_server_job_alone_and_in_mix():
    jobs = [workloads.Job(2, 24, tc_potts_2d(3), 61, 120, q=3), workloads.Job(2, 24, 2.3, 62, 120),
            workloads.Job(3, 6, 1.8, 63, 100, q=5)]
    with binding.Server(0, 0) as srv:
        ids = [srv.submit(j) for j in jobs]
        while srv.stats()["queued"] or srv.stats()["running"]:
            srv.step(2.0)
        got = {i: srv.take(i) for i in ids}
    for jid, j in zip(ids, jobs):
        if j.q:
            ref, _ = oracle_potts(j.dim, j.L, j.q, 1.0, j.T, j.seed, j.n_updates)
        else:
            S = oracle.init_spins(j.dim, j.L, j.seed)
            ref = oracle.run(j.dim, j.L, oracle.threshold(1.0, j.T), j.seed, 0, j.n_updates, S)
        assert (as_array(got[jid]) == ref).all()
