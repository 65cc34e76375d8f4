"""The two single-lattice workloads as configured: square lattice L = 4096 at
T_c and simple-cubic L = 256 at T = 4.511528, each from its random start
through 10^3 thermalisation + 10^4 measured updates on one lattice, checked
segment-parallel against the CPU oracle.

The GPU keeps every record and checkpoints the spins at the start of each
segment of 10^3 updates and again a few updates into it.  Host threads (the
oracle is C called through ctypes, which releases the GIL) then
  * replay the first updates of every segment from its checkpoint and
    compare records and spins bit for bit (state = (spins, t) and the random
    stream is counter-based, so a segment replays from its checkpoint
    alone),
  * recount (B, M) of every checkpoint and compare them with the GPU's
    record of the update before it,
and the whole record stream is checked against the exact identity
|M_t - M_{t-1}| = 2 |C_t| of the Wolff flip (Section 2, step (iv)).
Run on the library's default path choice and on the LDS-resident path."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from paper_1110_0899_amd import binding, workloads

pytestmark = pytest.mark.gpu

WORKLOADS = [(2, 4096, workloads.TC_2D, 2), (3, 256, workloads.T_3D, 3)]
SEGMENT, N_SEGMENTS, WINDOW = 1000, 11, 6       # 10^3 + 10^4 updates


def as_array(rec):
    return np.stack([rec["bond_sum"], rec["mag"], rec["csize"]], axis=1)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available()
    binding.load()


@pytest.mark.parametrize("path", ["default", "lds"])
@pytest.mark.parametrize("dim,L,T,seed", WORKLOADS)
def test_configured_run_segment_parallel(dim, L, T, seed, path):
    print("case segments dim=%d L=%d path=%s" % (dim, L, path), flush=True)
    N = L ** dim
    thr = oracle.threshold(1.0, T)
    starts, windows, records = [], [], []
    with binding.Simulation(dim, L, 1.0, T, seed) as sim:
        if path == "lds":
            sim.set_path(binding.PATH_LDS)
        for k in range(N_SEGMENTS):
            starts.append(sim.spins())
            sim.run(WINDOW)
            sim.synchronize()
            windows.append(sim.spins())
            sim.run(SEGMENT - WINDOW)
            records.append(as_array(sim.observables()))
        assert sim.info().t == SEGMENT * N_SEGMENTS
        final = sim.spins()
    rec = np.concatenate(records)
    assert rec.shape == (SEGMENT * N_SEGMENTS, 3)

    # the exact magnetisation identity over all 11 000 records
    S0 = oracle.init_spins(dim, L, seed)
    assert (starts[0] == S0).all()
    B0, M0 = oracle.observables(dim, L, S0)
    mags = np.concatenate([[M0], rec[:, 1]])
    assert (np.abs(np.diff(mags)) == 2 * rec[:, 2]).all()

    def replay(k):
        S = starts[k].copy()
        t0 = k * SEGMENT
        ref = oracle.run(dim, L, thr, seed, t0, WINDOW, S)
        ok_rec = bool((ref == rec[t0:t0 + WINDOW]).all())
        ok_spins = bool((S == windows[k]).all())
        # the checkpoint against the record of the update before it
        ckpt = starts[k + 1] if k + 1 < N_SEGMENTS else final
        B, M = oracle.observables(dim, L, ckpt)
        last = rec[t0 + SEGMENT - 1]
        ok_ckpt = (B, M) == (int(last[0]), int(last[1]))
        return k, ok_rec, ok_spins, ok_ckpt

    with ThreadPoolExecutor(max_workers=N_SEGMENTS) as ex:
        results = list(ex.map(replay, range(N_SEGMENTS)))
    for k, ok_rec, ok_spins, ok_ckpt in results:
        assert ok_rec, "segment %d: records differ from the oracle" % k
        assert ok_spins, "segment %d: spins differ from the oracle" % k
        assert ok_ckpt, "segment %d: checkpoint (B, M) differs from the record stream" % k
