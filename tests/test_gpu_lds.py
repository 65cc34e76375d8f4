"""The LDS-resident growth path (the lattice as bits in the LDS of one or
several workgroups, slabs of whole rows / planes) against the CPU oracle,
bit for bit: records after every update and the final spins; one workgroup
and many slabs (the slab size lowered so that small lattices split), cold
lattices whose frontier overflows the LDS ring and crosses slab boundaries
many times, measurement on and off, switches to and from the other paths,
resume from a checkpoint at an earlier update index, and the benchmarked
sizes."""
import numpy as np
import pytest
import torch

import oracle
from paper_1110_0899_amd import binding, workloads

pytestmark = pytest.mark.gpu

TC2, T3 = workloads.TC_2D, workloads.T_3D


def as_array(rec):
    return np.stack([rec["bond_sum"], rec["mag"], rec["csize"]], axis=1)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available()
    binding.load()


def run_lds(dim, L, T, seed, n, slab_bits=None, measure=True, start=None, t0=0):
    print("case lds dim=%d L=%d T=%.4f seed=%d n=%d slab=%s measure=%d start=%s"
          % (dim, L, T, seed, n, slab_bits, measure, start is not None), flush=True)
    with binding.Simulation(dim, L, 1.0, T, seed) as sim:
        if slab_bits:
            sim.set_lds_slab(slab_bits)
        sim.set_path(binding.PATH_LDS)
        sim.set_measure(measure)
        if start is not None:
            sim.set_spins(start, t0)
        sim.run(n)
        return as_array(sim.observables()), sim.spins()


def check(dim, L, T, seed, n, slab_bits=None, measure=True, start=None, t0=0):
    got, S = run_lds(dim, L, T, seed, n, slab_bits, measure, start, t0)
    S0 = oracle.init_spins(dim, L, seed) if start is None else start.copy()
    ref = oracle.run(dim, L, oracle.threshold(1.0, T), seed, t0, n, S0)
    cols = slice(0, 3) if measure else slice(1, 3)
    bad = np.nonzero((got[:, cols] != ref[:, cols]).any(axis=1))[0]
    assert bad.size == 0, "first mismatch at update %d: %s vs %s" % (bad[0], got[bad[0]], ref[bad[0]])
    if not measure:
        assert (got[:, 0] == binding.NOT_MEASURED).all()
    assert (S == S0).all()
    return ref


ONE_WG = [
    (2, 2, 2.0, 300), (2, 3, TC2, 300), (2, 17, 1.8, 300), (2, 32, TC2, 2000), (2, 64, TC2, 300),
    (2, 100, 2.6, 200), (3, 2, T3, 300), (3, 3, 4.0, 300), (3, 8, T3, 300), (3, 13, 4.7, 200),
    (3, 32, T3, 100), (2, 16, 2.0, 300), (2, 48, 2.2, 200), (3, 16, 4.0, 200), (3, 48, T3, 60),
]


@pytest.mark.parametrize("dim,L,T,n", ONE_WG)
def test_one_workgroup(dim, L, T, n):
    check(dim, L, T, 200 + L, n)


# (dim, L, T, n, slab_bits): the slab count is 2..16
SLABS = [
    (2, 64, TC2, 300, 2048), (2, 64, TC2, 300, 1024), (2, 48, 2.2, 300, 1024),
    (2, 37, TC2, 300, 1024), (2, 100, 2.0, 120, 1024), (3, 16, T3, 200, 1024),
    (3, 9, 4.2, 300, 1024), (3, 20, 4.0, 100, 2048), (2, 200, TC2, 60, 1024),
]


@pytest.mark.parametrize("dim,L,T,n,slab", SLABS)
@pytest.mark.parametrize("measure", [True, False])
def test_slabs(dim, L, T, n, slab, measure):
    check(dim, L, T, 300 + L, n, slab, measure)


@pytest.mark.parametrize("split", [False, True])
def test_cold_lattices_cross_slabs_and_overflow(split):
    # ordered start below T_c: clusters of most of the lattice, frontiers far
    # beyond the LDS ring, and (split) many crossings per update: the
    # smallest slab that keeps at most 64 slabs of whole rows / planes
    # (64, 40 and 32 slabs here)
    for dim, L, T, n, small in [(2, 256, 1.5, 20, 1024), (3, 40, 3.0, 12, 4096),
                                (2, 512, 1.8, 6, 8192)]:
        N = L ** dim
        ref = check(dim, L, T, 77, n, small if split else None, True, np.ones(N, dtype=np.int8))
        assert ref[:, 2].max() > N // 2


def test_special_cases():
    for slab in (None, 1024):
        got, _ = run_lds(2, 64, 1e30, 3, 200, slab)
        assert (got[:, 2] == 1).all()
        start = np.ones(216, dtype=np.int8)
        got, _ = run_lds(3, 6, 1e-3, 4, 10, slab, True, start)
        assert (got[:, 2] == 216).all() and (got[:, 0] == 3 * 216).all()


def test_path_switches_and_resume():
    dim, L, T, seed = 2, 64, TC2, 91
    ref_all = oracle.run(dim, L, oracle.threshold(1.0, T), seed, 0, 400,
                         oracle.init_spins(dim, L, seed))
    with binding.Simulation(dim, L, 1.0, T, seed) as sim:
        sim.set_lds_slab(1024)
        parts = []
        for path, n in [(binding.PATH_LDS, 60), (binding.PATH_SINGLE, 70), (binding.PATH_LDS, 50),
                        (binding.PATH_TEAM, 40), (binding.PATH_LDS, 80)]:
            sim.set_path(path, 8)
            sim.run(n)
            parts.append(as_array(sim.observables()))
        got = np.concatenate(parts)
        mid = sim.spins()
        t_mid = sim.info().t
        # rewind to an earlier checkpoint and replay on the LDS path
        S100 = oracle.init_spins(dim, L, seed)
        oracle.run(dim, L, oracle.threshold(1.0, T), seed, 0, 100, S100)
        sim.set_spins(S100, 100)
        sim.set_path(binding.PATH_LDS)
        sim.run(200)
        again = as_array(sim.observables())
    assert (got == ref_all[:300]).all()
    assert t_mid == 300
    assert (again == ref_all[100:300]).all()
    assert mid is not None


def test_graph_free_chunks_and_abort():
    # many launches (the chunk rule) and a stop request on the LDS path
    dim, L, T, seed = 2, 256, TC2, 93
    with binding.Simulation(dim, L, 1.0, T, seed) as sim:
        sim.set_path(binding.PATH_LDS)
        sim.run(200000)
        sim.abort()
        with pytest.raises(binding.WolffError) as e:
            sim.synchronize()
        assert e.value.code == binding.EABORTED
        k = sim.info().t
        got = as_array(sim.observables())
        S = sim.spins()
        sim.run(5)
        after = as_array(sim.observables())
    assert 0 <= k < 200000 and len(got) == k
    S_ref = oracle.init_spins(dim, L, seed)
    ref = oracle.run(dim, L, oracle.threshold(1.0, T), seed, 0, k + 5, S_ref)
    assert (got == ref[:k]).all()
    assert (after == ref[k:]).all()
    assert S is not None


@pytest.mark.parametrize("dim,L,T,seed", [(2, 4096, TC2, 2), (3, 256, T3, 3)])
def test_full_size_windows(dim, L, T, seed):
    # the benchmarked lattices on 16 slabs: the random start, the ordered
    # start (lattice-scale clusters), and a thermalised window
    thr = oracle.threshold(1.0, T)
    N = L ** dim
    print("case lds full size dim=%d L=%d" % (dim, L), flush=True)
    with binding.Simulation(dim, L, 1.0, T, seed) as sim:
        sim.set_path(binding.PATH_LDS)
        sim.run(6)
        got = as_array(sim.observables())
        S = oracle.init_spins(dim, L, seed)
        ref = oracle.run(dim, L, thr, seed, 0, 6, S)
        assert (got == ref).all()
        assert (sim.spins() == S).all()
        sim.set_spins(np.ones(N, dtype=np.int8), 0)
        sim.run(300 if dim == 2 else 1000)
        sim.observables()
        S = sim.spins()
        t = sim.info().t
        sim.run(8)
        got = as_array(sim.observables())
        ref = oracle.run(dim, L, thr, seed, t, 8, S)
        assert (got == ref).all()
        assert (sim.spins() == S).all()
