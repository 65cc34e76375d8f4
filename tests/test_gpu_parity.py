"""GPU path against the CPU oracle, bit for bit: records (B, M, |C|) after
every update and the final spins, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_1110_0899_amd import binding, workloads

pytestmark = pytest.mark.gpu

TC2, T3 = workloads.TC_2D, workloads.T_3D


def as_array(rec):
    return np.stack([rec["bond_sum"], rec["mag"], rec["csize"]], axis=1)


def oracle_series(dim, L, T, seed, n, t0=0, S=None):
    thr = oracle.threshold(1.0, T)
    if S is None:
        S = oracle.init_spins(dim, L, seed)
    rec = oracle.run(dim, L, thr, seed, t0, n, S)
    return rec, S


def gpu_series(dim, L, T, seed, n, path=binding.PATH_AUTO, team=0, measure=True):
    print("case dim=%d L=%d T=%.6f seed=%d n=%d path=%d team=%d" % (dim, L, T, seed, n, path, team),
          flush=True)
    with binding.Simulation(dim, L, 1.0, T, seed) as sim:
        sim.set_path(path, team)
        sim.set_measure(measure)
        sim.run(n)
        rec = sim.observables()
        S = sim.spins()
        info = sim.info()
    return as_array(rec), S, info


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available()
    binding.load()


def test_threshold_matches_oracle():
    for T in (TC2, T3, 2.0, 2.6, 4.3, 4.7, 1e-3, 1e6):
        with binding.Simulation(2, 4, 1.0, T, 1) as sim:
            assert sim.info().threshold == oracle.threshold(1.0, T)


def test_initial_state_matches_oracle():
    for dim, L, seed in [(2, 32, 1), (2, 33, 9), (3, 8, 3), (3, 5, 4), (2, 1000, 5)]:
        with binding.Simulation(dim, L, 1.0, TC2, seed) as sim:
            S = sim.spins()
            info = sim.info()
        ref = oracle.init_spins(dim, L, seed)
        assert (S == ref).all()
        B, M = oracle.observables(dim, L, ref)
        assert info.mag == M and info.bond_sum == B


@pytest.mark.parametrize("dim,L,seed", [(2, 3, 103), (2, 5, 7), (3, 3, 11), (2, 33, 9)])
def test_fresh_handle_state_before_any_copy(dim, L, seed):
    # the observables of a fresh handle are those of the lattice its init
    # kernel wrote: read them, and one update, before any spin copy (a copy
    # synchronises the device and could hide a fill that is not ordered on
    # the handle's stream)
    T = TC2 if dim == 2 else T3
    print("case fresh dim=%d L=%d seed=%d" % (dim, L, seed), flush=True)
    with binding.Simulation(dim, L, 1.0, T, seed) as sim:
        info = sim.info()
        sim.run(1)
        rec = as_array(sim.observables())
    B, M = oracle.observables(dim, L, oracle.init_spins(dim, L, seed))
    assert (info.mag, info.bond_sum) == (M, B)
    ref, _ = oracle_series(dim, L, T, seed, 1)
    assert (rec == ref).all()


def test_c1_full_run_single_path():
    c = workloads.C1
    got, S, info = gpu_series(2, c["L"], c["T"], c["seed"], c["n_meas"], binding.PATH_SINGLE)
    ref, Sref = oracle_series(2, c["L"], c["T"], c["seed"], c["n_meas"])
    assert got.shape == ref.shape
    bad = np.nonzero((got != ref).any(axis=1))[0]
    assert bad.size == 0, "first mismatch at update %d: %s vs %s" % (bad[0], got[bad[0]], ref[bad[0]])
    assert (S == Sref).all()
    assert info.t == c["n_meas"]


SMALL_CASES = [
    (2, 2, 2.0, 300), (2, 3, TC2, 300), (2, 17, 1.8, 300), (2, 64, TC2, 300), (2, 100, 2.6, 200),
    (3, 2, T3, 300), (3, 3, 4.0, 300), (3, 8, T3, 300), (3, 13, 4.7, 200), (3, 32, T3, 100),
    # tiled storage (L a multiple of 16), incl. tile counts that are not powers of two
    (2, 16, 2.0, 300), (2, 48, 2.2, 200), (3, 16, 4.0, 200), (3, 48, T3, 60),
]


def check_small(path, dim, L, T, n):
    seed = 100 + L
    got, S, _ = gpu_series(dim, L, T, seed, n, path, 8)
    ref, Sref = oracle_series(dim, L, T, seed, n)
    bad = np.nonzero((got != ref).any(axis=1))[0]
    assert bad.size == 0, "first mismatch at update %d: %s vs %s" % (bad[0], got[bad[0]], ref[bad[0]])
    assert (S == Sref).all()


def check_cold(path):
    # T well below T_c from the ordered state: clusters cover most of the
    # lattice, the frontier outgrows the LDS ring and the overflow stack /
    # global queue is used.
    # (L=512 / 3D L=64 have more sites than their member lists hold: clusters
    # above N/4 take the full-lattice measurement and tag clearing)
    for dim, L, T, n in [(2, 256, 1.5, 30), (3, 40, 3.0, 20), (2, 512, 1.8, 12), (3, 64, 3.5, 8)]:
        N = L ** dim
        start = np.ones(N, dtype=np.int8)
        print("case cold dim=%d L=%d T=%.3f path=%d" % (dim, L, T, path), flush=True)
        with binding.Simulation(dim, L, 1.0, T, 77) as sim:
            sim.set_path(path, 32)
            sim.set_spins(start, 0)
            sim.run(n)
            got = as_array(sim.observables())
            S = sim.spins()
        ref, Sref = oracle_series(dim, L, T, 77, n, S=start.copy())
        assert (got == ref).all()
        assert (S == Sref).all()
        assert ref[:, 2].max() > N // 2


def test_update_only_mode():
    got, S, _ = gpu_series(2, 32, TC2, 5, 500, binding.PATH_SINGLE, measure=False)
    ref, Sref = oracle_series(2, 32, TC2, 5, 500)
    assert (got[:, 0] == binding.NOT_MEASURED).all()
    assert (got[:, 1:] == ref[:, 1:]).all()
    assert (S == Sref).all()
    got, S, _ = gpu_series(3, 8, T3, 5, 200, binding.PATH_TEAM, 8, measure=False)
    ref, Sref = oracle_series(3, 8, T3, 5, 200)
    assert (got[:, 0] == binding.NOT_MEASURED).all()
    assert (got[:, 1:] == ref[:, 1:]).all()


def test_split_runs_and_resume():
    dim, L, T, seed = 2, 48, TC2, 31
    ref, Sref = oracle_series(dim, L, T, seed, 600)
    with binding.Simulation(dim, L, 1.0, T, seed) as sim:
        sim.run(100)
        sim.run(150)
        a = as_array(sim.observables())
        mid = sim.spins()
        sim.run(50)
        b = as_array(sim.observables())
    assert (np.concatenate([a, b]) == ref[:300]).all()
    # resume in a fresh handle from the checkpoint (spins, t)
    with binding.Simulation(dim, L, 1.0, T, 999) as sim2:
        pass
    with binding.Simulation(dim, L, 1.0, T, seed) as sim3:
        sim3.set_spins(mid, 250)
        sim3.run(350)
        c = as_array(sim3.observables())
        assert (c == ref[250:]).all()
        assert (sim3.spins() == Sref).all()


def test_range_error():
    with binding.Simulation(2, 4, 1.0, TC2, 1) as sim:
        sim.set_spins(np.ones(16, dtype=np.int8), 0xFFFFFFFE - 3)
        sim.run(3)
        with pytest.raises(binding.WolffError) as e:
            sim.run(2)
        assert e.value.code == binding.ERANGE


def test_special_cases():
    # T -> infinity: no active bond, |C| = 1
    got, _, _ = gpu_series(2, 16, 1e30, 3, 200)
    assert (got[:, 2] == 1).all()
    # T -> 0 from all up: the cluster is the whole lattice
    with binding.Simulation(3, 6, 1.0, 1e-3, 4) as sim:
        sim.set_spins(np.ones(216, dtype=np.int8), 0)
        sim.run(10)
        got = as_array(sim.observables())
    assert (got[:, 2] == 216).all() and (got[:, 0] == 3 * 216).all()


@pytest.mark.parametrize("lds", [True, False])
def test_batch_matches_oracle(lds):
    # lds: these lattices run on the batched LDS path, in both LDS-size
    # classes (square L = 600 and cubic L = 70 need more than 8 KiB
    # of LDS); off: all on the one-workgroup kernel
    jobs = [workloads.Job(2, 32, TC2, 11, 400), workloads.Job(3, 8, T3, 12, 300),
            workloads.Job(2, 17, 2.5, 13, 350), workloads.Job(2, 128, 2.0, 14, 60),
            workloads.Job(3, 5, 4.0, 15, 500), workloads.Job(2, 2, 1.0, 16, 100),
            workloads.Job(2, 600, TC2, 17, 30), workloads.Job(3, 70, T3, 18, 40)]
    print("case batch lds=%d" % lds, flush=True)
    with binding.Batch(jobs) as b:
        b.set_lds(lds)
        b.run(150)                      # one launch, at most 150 updates each
        b.run()                          # the rest
        for i, j in enumerate(jobs):
            got = as_array(b.records(i))
            ref, Sref = oracle_series(j.dim, j.L, j.T, j.seed, j.n_updates)
            assert (got == ref).all(), i
            assert (b.spins(i) == Sref).all(), i


# ---- one-workgroup path
@pytest.mark.parametrize("dim,L,T,n", SMALL_CASES)
def test_small_lattices_single(dim, L, T, n):
    check_small(binding.PATH_SINGLE, dim, L, T, n)


def test_cold_lattice_single():
    check_cold(binding.PATH_SINGLE)


# ---- multi-workgroup team path
def test_c1_team_path():
    c = workloads.C1
    n = 2000
    got, S, _ = gpu_series(2, c["L"], c["T"], c["seed"], n, binding.PATH_TEAM, 16)
    ref, Sref = oracle_series(2, c["L"], c["T"], c["seed"], n)
    assert (got == ref).all()
    assert (S == Sref).all()


@pytest.mark.parametrize("dim,L,T,n", SMALL_CASES)
def test_small_lattices_team(dim, L, T, n):
    check_small(binding.PATH_TEAM, dim, L, T, n)


def test_cold_lattice_team():
    check_cold(binding.PATH_TEAM)


# ---- captured graphs
@pytest.mark.parametrize("measure", [True, False])
def test_team_graph_replays_match_oracle(measure):
    dim, L, T, seed = 2, 40, TC2, 44
    ref, Sref = oracle_series(dim, L, T, seed, 120)
    with binding.Simulation(dim, L, 1.0, T, seed) as sim:
        sim.set_path(binding.PATH_TEAM, 8)
        sim.set_measure(measure)
        sim.set_graph(16)
        got = []
        for n in (37, 40, 16, 27):          # replays + eager remainders, synchronised in between
            sim.run(n)
            got.append(as_array(sim.observables()))
            sim.synchronize()
        got = np.concatenate(got)
        S = sim.spins()
    cols = slice(0, 3) if measure else slice(1, 3)
    assert (got[:, cols] == ref[:, cols]).all()
    assert (S == Sref).all()


def test_batch_graph_replays_match_oracle():
    # graphs serve the one-workgroup kernel's launches
    jobs = [workloads.Job(2, 24, TC2, 61, 90), workloads.Job(3, 6, T3, 62, 90)]
    with binding.Batch(jobs) as b:
        b.set_lds(False)
        b.set_graph(True)
        for _ in range(6):                 # the same captured launch replayed 6 times
            b.run(15)
            b.progress(0)
        for i, j in enumerate(jobs):
            ref, Sref = oracle_series(j.dim, j.L, j.T, j.seed, j.n_updates)
            assert (as_array(b.records(i)) == ref).all()
            assert (b.spins(i) == Sref).all()


def test_measure_switch_midway():
    # measured, update-only, measured again: the energy after the switch back
    # must come from a fresh lattice pass, not from a stale running sum
    dim, L, T, seed = 2, 64, TC2, 71
    ref, Sref = oracle_series(dim, L, T, seed, 300)
    for path in (binding.PATH_SINGLE, binding.PATH_TEAM):
        with binding.Simulation(dim, L, 1.0, T, seed) as sim:
            sim.set_path(path, 8)
            sim.run(100)
            sim.set_measure(False)
            sim.run(100)
            sim.set_measure(True)
            sim.run(100)
            got = as_array(sim.observables())
        assert (got[:100] == ref[:100]).all()
        assert (got[100:200, 0] == binding.NOT_MEASURED).all()
        assert (got[100:200, 1:] == ref[100:200, 1:]).all()
        assert (got[200:] == ref[200:]).all(), path


def test_path_switch_after_tagged_updates():
    # measured one-workgroup updates leave member tags in the lattice; the
    # team path must see plain spins, and both must stay on the oracle's
    # trajectory across several epochs of tags (more than 32 updates)
    dim, L, T, seed = 2, 48, TC2, 83
    ref, Sref = oracle_series(dim, L, T, seed, 230)
    with binding.Simulation(dim, L, 1.0, T, seed) as sim:
        sim.set_path(binding.PATH_SINGLE)
        sim.run(70)
        sim.set_path(binding.PATH_TEAM, 8)
        sim.run(50)
        sim.set_path(binding.PATH_SINGLE)
        sim.run(40)
        S_mid = sim.spins()
        sim.set_measure(False)
        sim.run(30)
        sim.set_measure(True)
        sim.set_path(binding.PATH_TEAM, 8)
        sim.run(40)
        got = as_array(sim.observables())
        S = sim.spins()
    assert set(np.unique(S_mid)) <= {-1, 1}
    assert (got[:160] == ref[:160]).all()
    assert (got[160:190, 1:] == ref[160:190, 1:]).all()
    assert (got[190:] == ref[190:]).all()
    assert (S == Sref).all()


@pytest.mark.parametrize("dim,L,T", [(2, 64, TC2), (3, 16, T3), (2, 32, 1.5), (3, 12, 3.0)])
def test_long_measured_run_single(dim, L, T):
    # many epochs of member tags: the running bond sum is cross-checked
    # against a lattice recount every 32 updates inside the kernel
    n = 700
    got, S, _ = gpu_series(dim, L, T, 97, n, binding.PATH_SINGLE)
    ref, Sref = oracle_series(dim, L, T, 97, n)
    assert (got == ref).all()
    assert (S == Sref).all()


def test_auto_path_follows_cost():
    # AUTO starts a large lattice on the team path; it then weighs the paths'
    # costs from the returned cluster sizes.  Small clusters of a measured
    # Potts lattice stay on the team path (one workgroup would recount the
    # lattice after each update); "update only" they move to one workgroup,
    # and back when measurement returns.  The records stay on the oracle's
    # trajectory throughout.
    dim, L, q, T, seed, n = 2, 1024, 3, 2.0, 29, 30
    thr = oracle.potts_threshold(1.0, T)
    C = oracle.potts_init(dim, L, q, seed)
    ref = oracle.potts_run(dim, L, q, thr, seed, 0, 3 * n, C)
    with binding.Simulation(dim, L, 1.0, T, seed, q=q) as sim:
        assert sim.info().path == binding.PATH_TEAM
        sim.run(n)
        got1 = as_array(sim.observables())
        assert sim.info().path == binding.PATH_TEAM
        sim.set_measure(False)
        assert sim.info().path == binding.PATH_SINGLE
        sim.run(n)
        got2 = as_array(sim.observables())
        sim.set_measure(True)
        assert sim.info().path == binding.PATH_TEAM
        sim.run(n)
        got3 = as_array(sim.observables())
        got = np.concatenate([got1, got2, got3])
        assert (sim.spins() == C).all()
    assert (got[:n] == ref[:n]).all()
    assert (got[n:2 * n, 1:] == ref[n:2 * n, 1:]).all()
    assert (got[2 * n:] == ref[2 * n:]).all()


def test_auto_path_picks_one_workgroup_for_mid_size_clusters():
    # square lattice L = 1024 at T_c with measurement, from the ordered
    # state, its LDS slabs lowered so that the lattice would take 16 of
    # them (2^20 sites, below the size from which AUTO takes a split LDS
    # lattice): the cost model chooses between the other two paths, and
    # once the clusters have relaxed to a few 1e5 sites (updates 20 to 40
    # of this seed) one workgroup is the cheaper one
    dim, L, T, seed = 2, 1024, TC2, 31
    thr = oracle.threshold(1.0, T)
    S = np.ones(L * L, dtype=np.int8)
    ref = oracle.run(dim, L, thr, seed, 0, 60, S)
    with binding.Simulation(dim, L, 1.0, T, seed) as sim:
        assert sim.info().path == binding.PATH_LDS           # one slab: the LDS path
        sim.set_lds_slab(1 << 16)
        sim.set_spins(np.ones(L * L, dtype=np.int8), 0)
        assert sim.info().path == binding.PATH_TEAM
        parts = []
        for _ in range(3):
            sim.run(20)
            parts.append(as_array(sim.observables()))
            if len(parts) == 2:
                assert sim.info().path == binding.PATH_SINGLE
        assert (sim.spins() == S).all()
    assert (np.concatenate(parts) == ref).all()


def test_auto_takes_two_slab_lattices_to_lds():
    # simple-cubic L = 128 (2^21 sites) needs two LDS slabs; AUTO takes the
    # LDS path for it, and its records and spins follow the oracle from the
    # random start and from the ordered start (lattice-scale clusters that
    # cross between the two slabs at every update)
    dim, L, T, seed = 3, 128, T3, 41
    thr = oracle.threshold(1.0, T)
    print("case auto two slabs 3D L=128", flush=True)
    for start, n in (("random", 20), ("ordered", 8)):
        S0 = oracle.init_spins(dim, L, seed) if start == "random" else np.ones(L ** dim, dtype=np.int8)
        ref = oracle.run(dim, L, thr, seed, 0, n, S0)
        with binding.Simulation(dim, L, 1.0, T, seed) as sim:
            if start == "ordered":
                sim.set_spins(np.ones(L ** dim, dtype=np.int8), 0)
            assert sim.info().path == binding.PATH_LDS
            sim.run(n)
            got = as_array(sim.observables())
            assert (sim.spins() == S0).all(), start
        assert (got == ref).all(), start


@pytest.mark.parametrize("wg,q", [(64, 64), (128, 128), (256, 2048), (512, 4096), (1024, 1024),
                                  (1024, 8192)])
def test_tile_sizes_single_and_batch(wg, q):
    # every workgroup size / ring size gives the oracle's records; the small
    # rings overflow to the global stack on the larger lattice
    cases = [(2, 48, TC2, 7, 80), (3, 12, T3, 8, 60)]
    for dim, L, T, seed, n in cases:
        print("case tiles wg=%d q=%d dim=%d L=%d" % (wg, q, dim, L), flush=True)
        ref, Sref = oracle_series(dim, L, T, seed, n)
        with binding.Simulation(dim, L, 1.0, T, seed) as sim:
            sim.set_path(binding.PATH_SINGLE)
            sim.set_tiles(wg, q)
            sim.run(n)
            assert (as_array(sim.observables()) == ref).all()
            assert (sim.spins() == Sref).all()
    jobs = [workloads.Job(d, L, T, seed, n) for d, L, T, seed, n in cases]
    with binding.Batch(jobs) as b:
        b.set_lds(False)                   # the tiles are the one-workgroup kernel's
        b.set_tiles(wg, q)
        b.run()
        for i, (d, L, T, seed, n) in enumerate(cases):
            ref, _ = oracle_series(d, L, T, seed, n)
            assert (as_array(b.records(i)) == ref).all()


def test_tile_sizes_rejected():
    with binding.Simulation(2, 16, 1.0, TC2, 1) as sim:
        for wg, q in [(1024, 16384), (100, 256), (256, 128), (256, 3000), (2048, 4096)]:
            with pytest.raises(binding.WolffError):
                sim.set_tiles(wg, q)
