"""The rest of the C ABI against the CPU oracle: a lattice on caller-owned
device buffers (wolff_create_ex, torch tensors) and the stop request
(wolff_abort, WOLFF_EABORTED), whose state after the stop must be the
oracle's after the updates that ran, with the handle still usable."""
import threading
import time

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


def tensors(N, cap, team=False):
    dev = torch.device("cuda:0")
    t = {"spins": torch.zeros((N + 3) // 4 * 4, dtype=torch.int8, device=dev),
         "overflow": torch.zeros(N, dtype=torch.int32, device=dev),
         "records": torch.zeros((cap, 3), dtype=torch.int64, device=dev)}
    if team:
        t["team_queue"] = torch.zeros(N, dtype=torch.int64, device=dev)
    return t


def addresses(t, cap, **extra):
    d = {k: v.data_ptr() for k, v in t.items()}
    d["record_capacity"] = cap
    d.update(extra)
    return d


@pytest.mark.parametrize("dim,L,T,path,team_queue", [
    (2, 48, TC2, binding.PATH_SINGLE, False), (2, 37, 2.2, binding.PATH_SINGLE, False),
    (3, 9, T3, binding.PATH_TEAM, True), (2, 40, TC2, binding.PATH_TEAM, False)])
def test_create_ex_on_torch_buffers(dim, L, T, path, team_queue):
    N = L ** dim
    n, cap, seed = 150, 400, 17
    print("case create_ex dim=%d L=%d path=%d" % (dim, L, path), flush=True)
    t = tensors(N, cap, team_queue)
    sim = binding.Simulation(dim, L, 1.0, T, seed, buffers=addresses(t, cap))
    try:
        sim.set_path(path, 8)
        sim.run(n)
        sim.synchronize()
        # the caller's tensors hold the lattice (site order, plain +-1) and the records
        S_dev = t["spins"][:N].cpu().numpy()
        rec_dev = t["records"][:n].cpu().numpy()
        got = as_array(sim.observables())
        S_ref = oracle.init_spins(dim, L, seed)
        ref = oracle.run(dim, L, oracle.threshold(1.0, T), seed, 0, n, S_ref)
        assert (got == ref).all()
        assert (rec_dev == ref).all()
        assert (S_dev == S_ref).all()
        assert (sim.spins() == S_ref).all()
        # more records than the buffer holds beside the pending ones: refused
        sim.run(cap - 10)
        with pytest.raises(binding.WolffError) as e:
            sim.run(20)
        assert e.value.code == binding.EINVAL
        sim.observables()
        sim.run(20)
        assert len(sim.observables()) == 20
    finally:
        sim.close()
    # the buffers stay the caller's
    assert t["spins"].is_cuda and t["records"].shape == (cap, 3)


def test_create_ex_keeps_callers_state():
    dim, L, T, seed, t0, n, cap = 2, 32, TC2, 5, 1234, 200, 256
    N = L * L
    S0 = oracle.init_spins(dim, L, 99)                 # some other state
    t = tensors(N, cap)
    t["spins"][:N] = torch.from_numpy(S0).cuda()
    with binding.Simulation(dim, L, 1.0, T, seed, buffers=addresses(t, cap, t0=t0)) as sim:
        info = sim.info()
        assert info.t == t0
        B, M = oracle.observables(dim, L, S0)
        assert (info.bond_sum, info.mag) == (B, M)
        sim.run(n)
        got = as_array(sim.observables())
        sim.synchronize()
        S_dev = t["spins"][:N].cpu().numpy()
    S = S0.copy()
    ref = oracle.run(dim, L, oracle.threshold(1.0, T), seed, t0, n, S)
    assert (got == ref).all()
    assert (S_dev == S).all()


def test_create_ex_rejects_bad_buffers():
    t = tensors(64, 8)
    for bad in ({"spins": 0}, {"record_capacity": 0}, {"overflow": t["overflow"].data_ptr() + 2},
                {"spins": t["spins"].data_ptr() + 4}):
        d = addresses(t, 8)
        d.update(bad)
        with pytest.raises(binding.WolffError) as e:
            binding.Simulation(2, 8, 1.0, TC2, 1, buffers=d)
        assert e.value.code == binding.EINVAL


@pytest.mark.parametrize("path", [binding.PATH_SINGLE, binding.PATH_TEAM])
def test_abort_stops_at_an_update_boundary(path):
    # a long run stopped right after it was enqueued: the state is the
    # oracle's after the updates that ran, and the handle carries on
    dim, L, T, seed, n = 2, 512, TC2, 41, 20000
    print("case abort path=%d" % path, flush=True)
    thr = oracle.threshold(1.0, T)
    with binding.Simulation(dim, L, 1.0, T, seed) as sim:
        sim.set_path(path, 16)
        sim.run(3)
        sim.synchronize()
        first = as_array(sim.observables())
        a = time.perf_counter()
        sim.run(n)
        sim.abort()
        with pytest.raises(binding.WolffError) as e:
            sim.synchronize()
        assert e.value.code == binding.EABORTED
        assert time.perf_counter() - a < 5.0
        info = sim.info()                              # reported once: no error now
        k = info.t - 3
        assert 0 <= k < n
        got = as_array(sim.observables())
        assert len(got) == k
        S = sim.spins()
        sim.run(5)                                     # usable again
        after = as_array(sim.observables())
        S_after = sim.spins()
    S_ref = oracle.init_spins(dim, L, seed)
    ref = oracle.run(dim, L, thr, seed, 0, 3 + k, S_ref)
    assert (first == ref[:3]).all()
    assert (got == ref[3:]).all()
    assert (S == S_ref).all()
    ref2 = oracle.run(dim, L, thr, seed, 3 + k, 5, S_ref)
    assert (after == ref2).all()
    assert (S_after == S_ref).all()


def test_abort_from_another_thread():
    dim, L, T, seed = 3, 64, T3, 43
    with binding.Simulation(dim, L, 1.0, T, seed) as sim:
        sim.set_path(binding.PATH_SINGLE)
        sim.run(200000)
        timer = threading.Timer(0.3, sim.abort)
        timer.start()
        with pytest.raises(binding.WolffError) as e:
            sim.synchronize()                          # blocks until the stop
        timer.join()
        assert e.value.code == binding.EABORTED
        t = sim.info().t
        assert 0 < t < 200000
        got = as_array(sim.observables())
        # the last few records against the oracle from the final state is not
        # possible without the state before them: check the invariant instead
        N = L ** dim
        B0, M0 = oracle.observables(dim, L, oracle.init_spins(dim, L, seed))
        dM = np.abs(np.diff(np.concatenate([[M0], got[:, 1]])))
        assert (dM == 2 * got[:, 2]).all()
        B, M = oracle.observables(dim, L, sim.spins())
        assert (got[-1, 0], got[-1, 1]) == (B, M)
        assert len(got) == t and (got[:, 2] >= 1).all() and (got[:, 2] <= N).all()


def test_abort_with_nothing_running_is_harmless():
    with binding.Simulation(2, 16, 1.0, TC2, 3) as sim:
        sim.run(10)
        sim.synchronize()
        sim.abort()
        sim.synchronize()                              # nothing was skipped: no error
        assert sim.info().t == 10
        sim.run(10)
        assert len(sim.observables()) == 20
