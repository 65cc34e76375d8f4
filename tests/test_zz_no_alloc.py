"""The no-allocation entry point (wolff_run_noalloc) against the entry point
it is a variant of: wolff_create_ex on caller-owned torch buffers, held on
the one-workgroup path, run and synchronised.  Two calls in a row share the
library's fixed device array, the second on a smaller lattice; both must
give the same records and final spins as the allocating path, bit for bit,
and the first also the CPU oracle's."""
import numpy as np
import pytest
import torch

import oracle
from paper_1110_0899_amd import binding, workloads

pytestmark = pytest.mark.gpu

TC2, T3 = workloads.TC_2D, workloads.T_3D
MAX_SITES = 1 << 20


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available()
    binding.load()


def reference(dim, L, T, seed, n, measure, start=None, t0=0):
    """Records and final spins through wolff_create_ex (the allocating path)."""
    N = L ** dim
    dev = torch.device("cuda:0")
    spins = torch.zeros((N + 3) // 4 * 4, dtype=torch.int8, device=dev)
    ov = torch.zeros(N, dtype=torch.int32, device=dev)
    rec = torch.zeros((n, 3), dtype=torch.int64, device=dev)
    bufs = {"spins": spins.data_ptr(), "overflow": ov.data_ptr(), "records": rec.data_ptr(),
            "record_capacity": n}
    if start is not None:
        spins[:N] = torch.from_numpy(start).to(dev)
        bufs["t0"] = t0
    torch.cuda.synchronize()            # the library's stream does not wait for torch's
    with binding.Simulation(dim, L, 1.0, T, seed, buffers=bufs) as sim:
        sim.set_path(binding.PATH_SINGLE)
        sim.set_measure(measure)
        sim.run(n)
        sim.synchronize()
        r = sim.observables()
        got = np.stack([r["bond_sum"], r["mag"], r["csize"]], axis=1)
    return got, spins[:N].cpu().numpy()


def noalloc(dim, L, T, seed, n, measure, start=None, t0=0, stream=None):
    N = L ** dim
    dev = torch.device("cuda:0")
    # buffers padded with a sentinel, to see that nothing is written past them
    spins = torch.full((N + 64,), 0x55, dtype=torch.int8, device=dev)
    rec = torch.full((n + 4, 3), -7, dtype=torch.int64, device=dev)
    if start is not None:
        spins[:N] = torch.from_numpy(start).to(dev)
    torch.cuda.synchronize()            # the fills are on torch's stream
    binding.run_noalloc(dim, L, 1.0, T, seed, spins.data_ptr(), n, rec.data_ptr(),
                        t0=t0 if start is not None else None, measure=measure, stream=stream)
    out = rec.cpu().numpy()
    S = spins.cpu().numpy()
    assert (out[n:] == -7).all() and (S[N:] == 0x55).all(), "write past the caller's buffers"
    return out[:n], S[:N]


@pytest.mark.parametrize("first,second", [
    ((2, 96, TC2, 11, 300, True), (2, 37, 2.2, 12, 200, True)),
    ((3, 24, T3, 13, 200, True), (2, 16, TC2, 14, 150, False)),
    ((2, 1024, TC2, 15, 20, True), (3, 9, 4.0, 16, 100, True)),
])
def test_two_calls_match_the_allocating_path(first, second):
    for k, (dim, L, T, seed, n, measure) in enumerate((first, second)):
        print("case noalloc call %d dim=%d L=%d n=%d measure=%d" % (k, dim, L, n, measure), flush=True)
        got, S = noalloc(dim, L, T, seed, n, measure)
        ref, S_ref = reference(dim, L, T, seed, n, measure)
        bad = np.nonzero((got != ref).any(axis=1))[0]
        assert bad.size == 0, "call %d: first mismatch at update %d: %s vs %s" % (
            k, bad[0], got[bad[0]], ref[bad[0]])
        assert (S == S_ref).all()
        if k == 0 and L ** dim <= 100000:
            S0 = oracle.init_spins(dim, L, seed)
            orc = oracle.run(dim, L, oracle.threshold(1.0, T), seed, 0, n, S0)
            cols = slice(0, 3) if measure else slice(1, 3)
            assert (got[:, cols] == orc[:, cols]).all()
            assert (S == S0).all()


def test_resume_from_a_checkpoint_and_a_torch_stream():
    dim, L, T, seed = 2, 45, TC2, 21
    S0 = oracle.init_spins(dim, L, seed)
    oracle.run(dim, L, oracle.threshold(1.0, T), seed, 0, 70, S0)    # S0 now at t = 70
    start = S0.copy()
    stream = torch.cuda.Stream()
    print("case noalloc resume t0=70 on a torch stream", flush=True)
    got, S = noalloc(dim, L, T, seed, 120, True, start=start, t0=70, stream=stream)
    ref, S_ref = reference(dim, L, T, seed, 120, True, start=start, t0=70)
    assert (got == ref).all() and (S == S_ref).all()
    orc = oracle.run(dim, L, oracle.threshold(1.0, T), seed, 70, 120, S0)
    assert (got == orc).all() and (S == S0).all()


def test_sizes_beyond_the_limit_are_rejected():
    dev = torch.device("cuda:0")
    spins = torch.zeros(16, dtype=torch.int8, device=dev)
    rec = torch.zeros((1, 3), dtype=torch.int64, device=dev)
    with pytest.raises(binding.WolffError) as e:
        binding.run_noalloc(2, 1025, 1.0, TC2, 1, spins.data_ptr(), 1, rec.data_ptr())
    assert e.value.code == binding.EINVAL
    with pytest.raises(binding.WolffError) as e:
        binding.run_noalloc(3, 102, 1.0, T3, 1, spins.data_ptr(), 1, rec.data_ptr())
    assert e.value.code == binding.EINVAL
    assert 1024 ** 2 <= MAX_SITES < 102 ** 3
