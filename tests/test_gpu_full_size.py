"""The benchmarked sizes (square lattice L = 4096, simple-cubic L = 256 at
their critical temperatures) in the launch configurations bench.py times,
against the CPU oracle on sampled windows of updates: a few updates from the
random start (small clusters) and a few from the ordered start (clusters that
fill most of the lattice, exercising the overflow stack and the team queue);
records and every spin compared bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_1110_0899_amd import binding, workloads

pytestmark = pytest.mark.gpu

SIZES = [(2, 4096, workloads.TC_2D, 2), (3, 256, workloads.T_3D, 3)]


def as_array(rec):
    return np.stack([rec["bond_sum"], rec["mag"], rec["csize"]], axis=1)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available()
    binding.load()


@pytest.mark.parametrize("dim,L,T,seed", SIZES)
def test_team_full_size_sampled(dim, L, T, seed):
    print("case full-size team dim=%d L=%d" % (dim, L), flush=True)
    thr = oracle.threshold(1.0, T)
    N = L ** dim
    with binding.Simulation(dim, L, 1.0, T, seed) as sim:
        # the default at these sizes is the LDS path (its full-size windows
        # are in test_gpu_lds.py); here the multi-workgroup team kernel
        assert sim.info().path == binding.PATH_LDS
        sim.set_path(binding.PATH_TEAM)
        sim.run(8)
        got = as_array(sim.observables())
        S = oracle.init_spins(dim, L, seed)
        ref = oracle.run(dim, L, thr, seed, 0, 8, S)
        assert (got == ref).all()
        assert (sim.spins() == S).all()
        # ordered start at a later update index
        sim.set_spins(np.ones(N, dtype=np.int8), 500)
        sim.run(2)
        got = as_array(sim.observables())
        S = np.ones(N, dtype=np.int8)
        ref = oracle.run(dim, L, thr, seed, 500, 2, S)
        assert (got == ref).all()
        assert ref[:, 2].max() > N // 4                           # a lattice-scale cluster
        assert (sim.spins() == S).all()


@pytest.mark.parametrize("dim,L,T,seed", SIZES)
def test_one_workgroup_full_size_sampled(dim, L, T, seed):
    # the one-workgroup path at its default tiles for these sizes (512
    # threads, 4096-entry ring), which the cost-based path choice takes for
    # the simple-cubic lattice at T_c
    print("case full-size one-workgroup dim=%d L=%d" % (dim, L), flush=True)
    thr = oracle.threshold(1.0, T)
    N = L ** dim
    with binding.Simulation(dim, L, 1.0, T, seed) as sim:
        sim.set_path(binding.PATH_SINGLE)
        sim.run(8)
        got = as_array(sim.observables())
        S = oracle.init_spins(dim, L, seed)
        ref = oracle.run(dim, L, thr, seed, 0, 8, S)
        assert (got == ref).all()
        assert (sim.spins() == S).all()
        sim.set_spins(np.ones(N, dtype=np.int8), 700)
        sim.run(2)
        got = as_array(sim.observables())
        S = np.ones(N, dtype=np.int8)
        ref = oracle.run(dim, L, thr, seed, 700, 2, S)
        assert (got == ref).all()
        assert ref[:, 2].max() > N // 4
        assert (sim.spins() == S).all()


@pytest.mark.parametrize("dim,L,T,seed", SIZES)
def test_batched_full_size_sampled(dim, L, T, seed):
    print("case full-size batch dim=%d L=%d" % (dim, L), flush=True)
    jobs = workloads.same_shape_jobs(dim, L, 2, 2)
    thr = oracle.threshold(1.0, T)
    with binding.Batch(jobs, start=1) as b:                      # ordered start, as bench.py
        b.set_tiles(512, 4096 if dim == 2 else 2048)
        b.run()
        for i, j in enumerate(jobs):
            S = np.ones(L ** dim, dtype=np.int8)
            ref = oracle.run(dim, L, thr, j.seed, 0, j.n_updates, S)
            assert (as_array(b.records(i)) == ref).all(), i
            assert (b.spins(i) == S).all(), i


@pytest.mark.parametrize("dim,L,T,seed", SIZES)
def test_plain_thermalised_window(dim, L, T, seed):
    # the headline's state: ordered start thermalised at T_c on the default
    # path, then a window of updates checkpointed and replayed by the oracle
    print("case full-size thermalised window dim=%d L=%d" % (dim, L), flush=True)
    thr = oracle.threshold(1.0, T)
    N = L ** dim
    n_therm, n_win = (300, 10) if dim == 2 else (1000, 10)
    with binding.Simulation(dim, L, 1.0, T, seed) as sim:
        sim.set_spins(np.ones(N, dtype=np.int8), 0)
        sim.run(n_therm)
        therm = as_array(sim.observables())
        S = sim.spins()
        t = sim.info().t
        sim.run(n_win)
        got = as_array(sim.observables())
        ref = oracle.run(dim, L, thr, seed, t, n_win, S)
        assert (got == ref).all()
        assert (sim.spins() == S).all()
    # invariants along the thermalisation run: |dM| = 2 |C| every update
    dM = np.abs(np.diff(np.concatenate([[N], therm[:, 1]])))
    assert (dM == 2 * therm[:, 2]).all()
    # the window is at equilibrium cluster sizes, not the ordering transient
    assert ref[:, 2].mean() < 0.5 * N
