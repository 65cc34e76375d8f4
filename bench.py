"""Benchmark of the Wolff single-cluster hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--legs plain2d,plain3d,...]

A step is one Wolff update of the whole hot path (seed draw, frontier growth
with bond activation, claim-and-flip, E/M measurement, record) on the
workload's lattice.  The headline workload is the square lattice L = 4096 at
T_c = 2/ln(1+sqrt 2) through the plain one-lattice launch path; the other
legs are reported under "extra": simple-cubic L = 256, both plain lattices
in "update only" mode, the L = 32 latency case with the oracle on all of it,
the batched persistent form on 2048 replicas of each lattice, the mixed
replica set, the serving stream, and a device-copy bandwidth for the
roofline.  Inputs are synthetic (seeded, no dataset).

Prints ONE JSON line.  `value` is added spins per second (sum of cluster
sizes over the timed updates / wall time between synchronisations).
`roofline` prices the dominant kernel (cluster growth) at the algorithmic
bytes per added spin (2d neighbour gathers + 8 B claim + 1 B flip + 8 B
queue write/read = 21 B in 2D, 23 B in 3D) against the 8 TB/s HBM peak,
timed per launch with HIP events on the stream the kernel runs on.
`cpu_baseline` times the CPU oracle (one core) on a bounded sample of the
same workload: it replays updates from the GPU's thermalised state, and its
records are compared with the GPU's for those updates.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_ADDED = {2: 21.0, 3: 23.0}
# Thermalisation of the headline lattices from the ordered state, whatever
# --warmup asks for: at least this many updates at T_c before the timed ones
# (the ordered start relaxes to the critical cluster-size level within a few
# hundred updates; a random start would take more than 10^6 at L = 4096)
MIN_THERM = {2: 1000, 3: 3000}
PAPER_CONTEXT = {
    "2d_L4096": "paper: 5.60x over one Xeon W3520 core (GTX 285, 83.95 ms/update incl. measurement)",
    "3d_L256": "paper: 7.90x over one Xeon W3520 core (GTX 285, 17.45 ms/update incl. measurement)",
}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    from paper_1110_0899_amd.profiling import kernel_source_sha as sha
    return sha()


def counter_summary(kernel: str, workload: str):
    """A committed rocprofv3 counter summary, if it was taken on the current
    kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "counters_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_sha") != kernel_source_sha():
        return None
    return d


def counter_traffic(kernel: str, workload: str, added_per_launch: float):
    """HBM bytes per launch of this run from the counter summary (else None):
    its bytes per added spin times the spins this run's launches add (a
    launch runs as many updates as fit its work budget, so launches of the
    counter run and of this run can differ in size)."""
    d = counter_summary(kernel, workload)
    if d is None or not d.get("hbm_bytes_per_added_spin"):
        return None
    return d["hbm_bytes_per_added_spin"] * added_per_launch


def ordered_start(n_sites: int) -> np.ndarray:
    return np.ones(n_sites, dtype=np.int8)


def plain_leg(binding, dim, L, T, seed, warmup, steps, start_ordered=True, measure=True,
              warm_sweeps=0.0, q=0, path=None):
    """Plain one-lattice path: warmup updates (and, with warm_sweeps, more
    until the flipped spins add up to that many lattice sweeps), then
    `steps` timed updates.  path: None for the library's cost-based choice,
    else a fixed binding.PATH_* value."""
    import torch
    sim = binding.Simulation(dim, L, 1.0, T, seed, q=q)
    if path is not None:
        sim.set_path(path)
    sim.set_measure(measure)
    if start_ordered:
        sim.set_spins(np.zeros(L ** dim, dtype=np.int8) if q else ordered_start(L ** dim), 0)
    t0 = time.time()
    sim.run(warmup)
    sim.synchronize()
    therm = sim.observables()
    therm_mean = float(therm["csize"][-200:].mean()) if len(therm) else 0.0
    if warm_sweeps:
        # small clusters: thermalise "update only" until the flipped spins add
        # up to warm_sweeps lattices
        sim.set_measure(False)
        flipped, last = 0, time.time()
        while flipped < warm_sweeps * L ** dim and warmup < 20_000_000:
            sim.run(50_000)
            flipped += int(sim.observables()["csize"].sum())
            warmup += 50_000
            if time.time() - last > 10.0:
                last = time.time()
                log("%dD L=%d T=%.4f: %d updates, %.2f sweeps flipped"
                    % (dim, L, T, warmup, flipped / L ** dim))
        sim.set_measure(measure)
        sim.run(100)
        sim.synchronize()
        sim.observables()
        warmup += 100
    log("%dD L=%d: %d warmup updates in %.1f s" % (dim, L, warmup, time.time() - t0))
    checkpoint = sim.spins()
    t_ckpt = sim.info().t
    path_timed = int(sim.info().path)        # the path the timed updates take
    sim.profile(True)
    torch.cuda.synchronize()
    sim.synchronize()
    a = time.perf_counter()
    sim.run(steps)
    sim.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - a
    rec = sim.observables()
    prof = sim.profile_read()
    info = sim.info()
    sim.close()
    added = int(rec["csize"].sum())
    grow_ms = prof["grow_ms"]
    achieved = BYTES_PER_ADDED[dim] * added / (grow_ms * 1e-3) / 1e9 if grow_ms > 0 else 0.0
    log("%dD L=%d: %d updates in %.2f s, <|C|>=%.0f, %.3e added/s, grow %.3f ms/launch"
        % (dim, L, steps, wall, added / max(steps, 1), added / wall,
           grow_ms / max(prof["grow_launches"], 1)))
    return {
        "dim": dim, "L": L, "T": T, "seed": seed, "q": q, "warmup": warmup, "steps": steps,
        "measurement": bool(measure),
        "wall_s": wall, "added": added, "added_per_s": added / wall,
        "updates_per_s": steps / wall, "mean_csize": added / max(steps, 1),
        "grow_ms": grow_ms, "grow_launches": prof["grow_launches"],
        "measure_ms": prof["measure_ms"], "measure_launches": prof["measure_launches"],
        "grow_GBs_algorithmic": achieved, "path": path_timed, "path_after": int(info.path),
        "records": rec, "checkpoint": checkpoint, "t_ckpt": t_ckpt,
        "therm_mean_csize": therm_mean,
    }


def batch_leg(binding, workloads, dim, L, n_rep, warmup, steps, wg=None, qe=None, potts_q=0):
    """Batched persistent form: n_rep same-shape replicas at T_c, one launch
    per run; warmup updates, then `steps` timed updates of every replica.
    Tile sizes (wg, LDS ring entries qe) come from the autotuner unless
    given; potts_q >= 2: the q-state Potts model."""
    jobs = workloads.same_shape_jobs(dim, L, n_rep, warmup + steps, q=potts_q)
    tuned = None
    if wg is None or qe is None:
        from paper_1110_0899_amd import autotune
        # tune on the replica count of the run: the best tiles depend on how
        # full the device is
        tjobs = workloads.same_shape_jobs(dim, L, n_rep, 16, q=potts_q)
        tuned = autotune.tune(tjobs, warm=8, timed=4, start=1, log=log)
        wg, qe = tuned["wg"], tuned["queue_entries"]
    b = binding.Batch(jobs, start=1)
    b.set_tiles(wg, qe)
    b.set_measure(True)
    t0 = time.time()
    b.run(warmup)
    b.last_ms()
    log("batch %dD L=%d x%d: %d warmup updates in %.1f s" % (dim, L, n_rep, warmup, time.time() - t0))
    for i in range(n_rep):
        b.records(i)
    a = time.perf_counter()
    b.run(steps)
    ms = b.last_ms()
    wall = time.perf_counter() - a
    added = 0
    for i in range(n_rep):
        added += int(b.records(i)["csize"].sum())
    b.close()
    kernel_s = ms * 1e-3
    log("batch %dD L=%d x%d: %d updates each in %.2f s (kernel %.2f s), %.3e added/s"
        % (dim, L, n_rep, steps, wall, kernel_s, added / kernel_s))
    return {
        "dim": dim, "L": L, "q": potts_q, "replicas": n_rep, "warmup": warmup, "steps": steps,
        "wg": wg, "queue_entries": qe, "wall_s": wall, "kernel_s": kernel_s, "added": added,
        "added_per_s": added / wall, "updates_per_s": n_rep * steps / wall,
        "mean_csize": added / (n_rep * steps),
        "kernel_GBs_algorithmic": BYTES_PER_ADDED[dim] * added / kernel_s / 1e9,
        "kernel_frac_of_hbm_peak": BYTES_PER_ADDED[dim] * added / kernel_s / 1e9 / HBM_PEAK_GBS,
        "tiles": "autotuner" if tuned else "fixed",
    }


def c1_leg(binding, workloads):
    """C1: square lattice L=32 at T_c from the random start, 10^4 measured
    updates; latency per update on the GPU, and the oracle on all of it
    (its records must equal the GPU's)."""
    import oracle
    c = workloads.C1
    n = c["n_meas"]
    with binding.Simulation(c["dim"], c["L"], 1.0, c["T"], c["seed"]) as sim:
        sim.run(1)
        sim.synchronize()
        sim.observables()
        a = time.perf_counter()
        sim.run(n)
        sim.synchronize()
        wall = time.perf_counter() - a
        rec = sim.observables()
        path = int(sim.info().path)
    S = oracle.init_spins(c["dim"], c["L"], c["seed"])
    thr = oracle.threshold(1.0, c["T"])
    oracle.run(c["dim"], c["L"], thr, c["seed"], 0, 1, S)
    a = time.perf_counter()
    ref = oracle.run(c["dim"], c["L"], thr, c["seed"], 1, n, S)
    cpu_s = time.perf_counter() - a
    got = np.stack([rec["bond_sum"], rec["mag"], rec["csize"]], axis=1)
    added = int(rec["csize"].sum())
    log("C1: %d updates, %.2f us/update on the GPU, oracle %.2f us/update, records match: %s"
        % (n, 1e6 * wall / n, 1e6 * cpu_s / n, bool((got == ref).all())))
    return {"updates": n, "gpu_us_per_update": 1e6 * wall / n, "gpu_added_per_s": added / wall,
            "oracle_us_per_update": 1e6 * cpu_s / n, "oracle_added_per_s": added / cpu_s,
            "oracle_cores": 1, "records_match_oracle": bool((got == ref).all()),
            "mean_csize": added / n, "path": path}


def c4_leg(binding, workloads, n_updates):
    """C4: the mixed replica set (256 square lattices L in {64..1024},
    T in [2.0, 2.6]; 64 simple-cubic L in {32, 64, 128}, T in [4.3, 4.7]),
    random starts, n_updates each in one persistent launch with measurement."""
    jobs = workloads.c4_jobs(n_updates)
    from paper_1110_0899_amd import autotune
    # the trial: 400 updates of every replica after 2000 from the random start.
    # The makespan is set by the largest replicas once their clusters have
    # grown; an early window (clusters still small) favours small workgroups
    # (128 threads: 17.7 s against 10.4 s with 256 over the whole run).
    # tiles of the one-workgroup kernel, tuned for each setting (with the LDS
    # classes it only runs the replicas that do not fit one workgroup's LDS)
    tuned = {lds: autotune.tune(workloads.c4_jobs(2400), warm=2000, timed=400, start=0, log=log,
                                lds=lds) for lds in (True, False)}

    def run(lds):
        b = binding.Batch(jobs, start=0)
        b.set_tiles(tuned[lds]["wg"], tuned[lds]["queue_entries"])
        b.set_measure(True)
        b.set_lds(lds)
        a = time.perf_counter()
        b.run()
        ms = b.last_ms()
        wall = time.perf_counter() - a
        per = [int(b.records(i)["csize"].sum()) for i in range(len(jobs))]
        b.close()
        if lds:
            # the replicas with the most work (sites flipped over the run)
            top = sorted(range(len(jobs)), key=lambda i: -per[i])[:5]
            heavy.extend({"dim": jobs[i].dim, "L": jobs[i].L, "T": round(jobs[i].T, 4),
                          "added": per[i]} for i in top)
        return wall, ms, sum(per)

    heavy = []

    # the replicas that fit one workgroup's LDS run on the batched LDS path;
    # the same set all on the one-workgroup kernel, for comparison
    wall, ms, added = run(True)
    wall_g, ms_g, added_g = run(False)
    assert added_g == added
    n_lds = sum(1 for j in jobs if (32 * -(-j.L // 32)) * j.L ** (j.dim - 1) <= (1 << 20))
    log("C4: %d replicas x %d updates (%d on the LDS path), makespan %.2f s (kernel %.2f s), "
        "%.3e added/s; all on the one-workgroup kernel: %.2f s"
        % (len(jobs), n_updates, n_lds, wall, ms * 1e-3, added / wall, wall_g))
    return {"replicas": len(jobs), "updates_each": n_updates, "makespan_s": wall,
            "kernel_s": ms * 1e-3, "added": added, "added_per_s": added / wall,
            "cluster_updates_per_s": len(jobs) * n_updates / wall,
            "replicas_on_lds_path": n_lds, "makespan_one_workgroup_kernel_s": wall_g,
            "wg": tuned[True]["wg"], "queue_entries": tuned[True]["queue_entries"],
            "heaviest_replicas": heavy,
            "wg_one_workgroup_kernel": tuned[False]["wg"],
            "queue_entries_one_workgroup_kernel": tuned[False]["queue_entries"]}


PAPER_TABLES = {  # ms per update at T_c on the paper's GTX 285 / one Xeon W3520 core (Tables 1-2):
    # (GPU update only, GPU + measurement, CPU update only, CPU + measurement)
    (2, 512): (7.634, 7.677, 4.151, 4.913), (2, 1024): (15.80, 16.10, 20.97, 24.19),
    (2, 2048): (33.02, 34.50, 87.59, 100.9), (2, 4096): (81.37, 83.95, 412.0, 470.9),
    (3, 64): (1.176, 1.378, 1.170, 1.947), (3, 128): (2.801, 3.483, 9.785, 15.76),
    (3, 256): (13.04, 17.45, 97.47, 137.9),
}


def sweep_point(binding, dim, L, T, seed, warmup, steps, start_ordered, cpu_seconds):
    """GPU ms per update in both modes (the same updates: state and random
    stream do not depend on the mode) and the oracle's ms per update with
    measurement, replayed from the GPU's state."""
    sweeps = 0.0 if start_ordered else 2.0
    m = plain_leg(binding, dim, L, T, seed, warmup, steps, start_ordered, measure=True,
                  warm_sweeps=sweeps)
    u = plain_leg(binding, dim, L, T, seed, warmup, steps, start_ordered, measure=False,
                  warm_sweeps=sweeps)
    cpu = cpu_baseline(m, cpu_seconds)
    gpu_ms = 1e3 * m["wall_s"] / steps
    cpu_ms = 1e3 * cpu["seconds"] / max(cpu["updates"], 1)
    return {"dim": dim, "L": L, "T": T, "start": "ordered" if start_ordered else "random",
            "warmup": m["warmup"], "steps": steps, "mean_csize": m["mean_csize"],
            "gpu_ms_update_only": 1e3 * u["wall_s"] / steps, "gpu_ms_measure": gpu_ms,
            "cpu_ms_measure": cpu_ms, "cpu_updates": cpu["updates"],
            "cpu_records_match": cpu["records_match_gpu"], "speedup_measure": cpu_ms / gpu_ms,
            "path": m["path"], "path_update_only": u["path"]}


def sizes_leg(binding, workloads, cpu_seconds):
    """The paper's size sweep (Tables 1-2) at T_c."""
    rows = []
    for dim, Ls, T, warm, steps in ((2, (512, 1024, 2048, 4096), workloads.TC_2D, 300, 300),
                                    (3, (64, 128, 256, 1024), workloads.T_3D, 1000, 1000)):
        for L in Ls:
            # 3D L=1024 (1 GiB of spins) is the size the paper expected to gain most
            r = sweep_point(binding, dim, L, T, 2 if dim == 2 else 3, warm, steps, True, cpu_seconds)
            if (dim, L) in PAPER_TABLES:
                r["paper_ms"] = dict(zip(("gpu_update_only", "gpu_measure", "cpu_update_only",
                                          "cpu_measure"), PAPER_TABLES[(dim, L)]))
            rows.append(r)
    return rows


def temps_leg(binding, workloads, cpu_seconds):
    """The paper's temperature sweep (Fig. 1): 2D L=4096 and 3D L=256 at
    T/T_c from 0.9 to 1.1; ordered start at and below T_c; above T_c a
    random start thermalised until the flipped spins add up to two lattices."""
    rows = []
    for dim, L, Tc, warm, steps in ((2, 4096, workloads.TC_2D, 100, 100),
                                    (3, 256, workloads.T_3D, 300, 300)):
        for f in (0.9, 0.95, 1.0, 1.05, 1.1):
            rows.append(sweep_point(binding, dim, L, Tc * f, 2 if dim == 2 else 3, warm, steps,
                                    f <= 1.0, cpu_seconds))
            rows[-1]["T_over_Tc"] = f
    return rows


def potts_leg(binding, workloads, args):
    """The q-state Potts extension (q = 3 at the square-lattice T_c): one
    lattice of L = 1024 with the oracle beside it and one of L = 4096 (both
    on the default growth path), and the batched form on --batch-replicas
    replicas of L = 4096 (tiles from the autotuner)."""
    q = 3
    T = workloads.potts_tc_2d(q)
    p = plain_leg(binding, 2, 1024, T, 2, 300, 300, q=q)
    cpu = cpu_baseline(p, args.sweep_cpu_seconds)
    p4 = plain_leg(binding, 2, 4096, T, 3, 200, 100, q=q)
    b = batch_leg(binding, workloads, 2, 4096, args.batch_replicas, args.batch_warmup,
                  args.batch_steps, potts_q=q)
    return {"q": q, "T": T,
            "plain_2d_L1024": {k: v for k, v in p.items() if k not in ("records", "checkpoint")},
            "plain_cpu_oracle": cpu,
            "plain_2d_L4096": {k: v for k, v in p4.items() if k not in ("records", "checkpoint")},
            "batch_2d_L4096": b}


def handoff_leg(reps=2000):
    """The fixed cost a host-started update would pay on this machine (the
    paper's hybrid start, Table 3): a synchronised device-to-host and
    host-to-device copy of a small frontier in pinned memory, and one kernel
    launch with a host synchronisation.  Plumbing only: no growth runs."""
    import torch
    dev = torch.device("cuda:0")
    out = {"round_trip_us": {}}
    for nbytes in (512, 4096, 65536):
        d = torch.zeros(nbytes // 4, dtype=torch.int32, device=dev)
        h = torch.zeros(nbytes // 4, dtype=torch.int32).pin_memory()
        for it in range(200 + reps):
            if it == 200:
                a = time.perf_counter()
            h.copy_(d, non_blocking=True)
            torch.cuda.synchronize()
            d.copy_(h, non_blocking=True)
            torch.cuda.synchronize()
        out["round_trip_us"][str(nbytes)] = (time.perf_counter() - a) / reps * 1e6
    x = torch.zeros(1, device=dev)
    for it in range(200 + reps):
        if it == 200:
            a = time.perf_counter()
        x.add_(1.0)
        torch.cuda.synchronize()
    out["launch_sync_us"] = (time.perf_counter() - a) / reps * 1e6
    log("hand-off: round trip %s us, launch + sync %.1f us"
        % (", ".join("%s B %.1f" % kv for kv in out["round_trip_us"].items()), out["launch_sync_us"]))
    return out


def copy_peak_gbs(reps=5):
    """Device-to-device copy bandwidth (read + write bytes / time), 2 GiB."""
    import torch
    n = 2 << 30
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * n * reps / el / 1e9


def serve_leg(binding, workloads, quantum_ms=5.0, n_jobs=2000, max_wall_s=30.0):
    """Serving form, measurement on: the loop's capacity from a saturated
    closed batch of stream-shaped jobs (twice its slots, all queued at once),
    then the Poisson stream at 1.2x that rate through the continuous-batching
    loop."""
    from paper_1110_0899_amd import serve
    with binding.Server() as probe:
        slots = int(probe.stats()["slots"])
    sample = workloads.c5_stream(n_jobs=2 * slots + 200, rate_per_s=1.0, seed=55)
    capinfo = serve.capacity(sample, quantum_ms, progress=log)
    cap = capinfo["jobs_per_s"]
    rate = 1.2 * cap
    stream = workloads.c5_stream(n_jobs=n_jobs, rate_per_s=rate)
    r = serve.run_stream(stream, quantum_ms=quantum_ms, max_wall_s=max_wall_s, progress=log)
    r.pop("records", None)
    r.pop("finish_s", None)
    last_arrival = max(j.arrival_s for j in stream if j.arrival_s <= max_wall_s)
    r.update({"capacity_jobs_per_s": cap, "capacity_estimate": capinfo,
              "arrival_rate_jobs_per_s": rate, "arrival_span_s": last_arrival,
              "quantum_ms": quantum_ms, "records": "E and M measured after every update"})
    log("serve: capacity %.1f jobs/s (closed batch of %d), stream at %.1f jobs/s over %.1f s: "
        "%d jobs, p50 %.3f s, p99 %.3f s, %.3e added/s"
        % (cap, capinfo["jobs"], rate, last_arrival, r["jobs"], r["p50_latency_s"],
           r["p99_latency_s"], r["added_per_s"]))
    return r


def cpu_baseline(leg, budget_s=15.0):
    """The CPU oracle (one core) replaying updates from the GPU checkpoint."""
    import oracle
    dim, L, T, seed, q = leg["dim"], leg["L"], leg["T"], leg["seed"], leg.get("q", 0)
    thr = oracle.potts_threshold(1.0, T) if q else oracle.threshold(1.0, T)
    S = leg["checkpoint"].copy()
    t = leg["t_ckpt"]
    gpu = leg["records"]
    done, added, match = 0, 0, True
    a = time.perf_counter()
    while done < len(gpu) and time.perf_counter() - a < budget_s:
        if q:
            rec = oracle.potts_run(dim, L, q, thr, seed, t + done, 1, S)
        else:
            rec = oracle.run(dim, L, thr, seed, t + done, 1, S)
        g = gpu[done]
        match &= (int(g["bond_sum"]), int(g["mag"]), int(g["csize"])) == tuple(int(v) for v in rec[0])
        added += int(rec[0, 2])
        done += 1
    el = time.perf_counter() - a
    log("cpu oracle: %d updates in %.1f s, %.3e added/s, records match GPU: %s"
        % (done, el, added / el, match))
    return {
        "value": added / el, "unit": "added spins/s", "cores": 1, "kind": "oracle",
        "sample": "%d consecutive updates of the %dD L=%d workload replayed from the GPU's "
                  "thermalised state (update %d on), full E/M recount per update"
                  % (done, dim, L, leg["t_ckpt"]),
        "updates": done, "seconds": el, "records_match_gpu": bool(match),
    }


def stats_counts(binding, workloads):
    """Counting build (libwolff_stats.so, loaded with WOLFF_LIBRARY=stats):
    the work and the global-memory bytes each hot kernel issues per added
    spin, on the benchmarked states: the headline lattice and the cubic
    L = 256 lattice thermalised on the default (LDS) path and on the team
    path, and 64 replicas of the batched form of each."""
    out = {}

    def per_spin(c):
        sites = max(c["sites"], 1)
        touched = c["read_bytes"] + c["write_bytes"] + c["atomic_bytes"]
        return {"counters": c, "bytes_touched_per_added_spin": touched / sites,
                "read_bytes_per_added_spin": c["read_bytes"] / sites,
                "write_bytes_per_added_spin": c["write_bytes"] / sites,
                "atomic_bytes_per_added_spin": c["atomic_bytes"] / sites,
                "philox_blocks_per_added_spin": c["philox"] / sites,
                "steps_per_update": c["steps"] / max(c["updates"], 1),
                "messages_per_added_spin": c["messages"] / sites,
                # LDS path, thread 0 of each workgroup: shader cycles per growth step
                "cycles_per_step": c["cycles_grow"] / max(c["steps"], 1),
                "cycles_expand_per_step": c["cycles_expand"] / max(c["steps"], 1),
                "cycles_publish_per_step": c["cycles_publish"] / max(c["steps"], 1),
                "send_steps_fraction": c["steps_send"] / max(c["steps"], 1),
                "cycles_send_per_send_step": c["cycles_send"] / max(c["steps_send"], 1),
                "idle_to_grow_cycles": c["cycles_idle"] / max(c["cycles_grow"], 1)}

    for dim, L, T, seed, warm, n in [(2, 4096, workloads.TC_2D, 2, 1000, 40),
                                     (3, 256, workloads.T_3D, 3, 3000, 200),
                                     (2, 1024, workloads.TC_2D, 4, 300, 200),
                                     (2, 32, workloads.TC_2D, 1, 300, 2000)]:
        for name, path in (("default", None), ("team", binding.PATH_TEAM)):
            if L < 4096 and L != 256 and path is not None:
                continue
            sim = binding.Simulation(dim, L, 1.0, T, seed)
            sim.set_spins(ordered_start(L ** dim), 0)
            sim.run(warm)
            sim.synchronize()
            sim.observables()
            if path is not None:
                sim.set_path(path)
            sim.stats(reset=True)
            sim.run(n)
            sim.synchronize()
            rec = sim.observables()
            c = sim.stats()
            path_used = int(sim.info().path)
            sim.close()
            r = per_spin(c)
            r["path"] = path_used
            r["updates"] = n
            r["added"] = int(rec["csize"].sum())
            out["%dd_L%d_%s" % (dim, L, name)] = r
            log("stats %dD L=%d %s (path %d): %.1f B touched / added spin, %.2f Philox blocks, "
                "%.0f steps / update, %.0f cycles / step (expand %.0f, publish %.0f; %.0f %% of "
                "steps send, %.0f cycles waiting for message credit per send step)"
                % (dim, L, name, path_used, r["bytes_touched_per_added_spin"],
                   r["philox_blocks_per_added_spin"], r["steps_per_update"], r["cycles_per_step"],
                   r["cycles_expand_per_step"], r["cycles_publish_per_step"],
                   100.0 * r["send_steps_fraction"], r["cycles_send_per_send_step"]))
    for dim, L, warm, n in [(2, 4096, 100, 8), (3, 256, 1000, 40)]:
        jobs = workloads.same_shape_jobs(dim, L, 64, warm + n)
        b = binding.Batch(jobs, start=1)
        b.run(warm)
        b.last_ms()
        b.stats(reset=True)
        b.run(n)
        c = b.stats()
        b.close()
        r = per_spin(c)
        out["batch_%dd_L%d_x64" % (dim, L)] = r
        log("stats batch %dD L=%d x64: %.1f B touched / added spin" % (dim, L, r["bytes_touched_per_added_spin"]))
    return out


def stats_leg():
    """stats_counts in a child process that loads the counting build."""
    import subprocess
    env = dict(os.environ, WOLFF_LIBRARY="stats")
    p = subprocess.run([sys.executable, os.path.abspath(__file__), "--profile-leg", "stats"],
                       env=env, capture_output=True, text=True)
    sys.stderr.write(p.stderr[-4000:])
    if p.returncode != 0:
        return {"error": "counting build run failed (rc %d)" % p.returncode}
    return json.loads(p.stdout.strip().splitlines()[-1])


def profile_only(args, binding, workloads):
    """One leg alone, for rocprofv3 runs (kernel trace or counters)."""
    import torch
    leg = args.profile_leg
    if leg == "copy":
        # calibration for the HBM counters: one device-to-device copy of 1 GiB
        n = 1 << 30
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        r = {"leg": "copy", "bytes_read": n, "bytes_written": n}
    elif leg in ("plain2d", "plain3d"):
        path = {"auto": None, "single": binding.PATH_SINGLE, "team": binding.PATH_TEAM,
                "lds": binding.PATH_LDS}[args.path]
        dim, L, T, seed = ((2, 4096, workloads.TC_2D, 2) if leg == "plain2d"
                           else (3, 256, workloads.T_3D, 3))
        r = plain_leg(binding, dim, L, T, seed, max(args.warmup, MIN_THERM[dim]), args.steps,
                      path=path)
    elif leg == "stats":
        r = stats_counts(binding, workloads)
    elif leg in ("batch2d", "batch3d"):
        wg, q = (int(v) for v in args.tiles.split(","))
        dim, L = (2, 4096) if leg == "batch2d" else (3, 256)
        r = batch_leg(binding, workloads, dim, L, args.batch_replicas, args.warmup,
                      args.batch_steps, wg=wg, qe=q)
    else:
        raise SystemExit("unknown leg %s" % leg)
    r = {k: v for k, v in r.items() if k not in ("records", "checkpoint")}
    r["leg"] = leg
    print(json.dumps(r), flush=True)


def build_parser() -> argparse.ArgumentParser:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000, help="timed updates of the headline leg")
    ap.add_argument("--warmup", type=int, default=1000, help="thermalisation updates")
    ap.add_argument("--legs", default="plain2d,plain3d,updateonly,c1,batch2d,batch3d,c4,serve,stats")
    ap.add_argument("--c4-updates", type=int, default=10000,
                    help="updates per replica of the mixed C4 batch")
    ap.add_argument("--batch-replicas", type=int, default=2048)
    ap.add_argument("--batch-steps", type=int, default=32)
    ap.add_argument("--batch-warmup", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--sweep-cpu-seconds", type=float, default=4.0,
                    help="oracle time per point of the sweeps (legs sizes, temps, potts, handoff; "
                         "run without plain2d, they print their own JSON line)")
    ap.add_argument("--tiles", default="512,2048",
                    help="workgroup size, LDS ring entries of a profiled batch leg (the full "
                         "benchmark takes them from the autotuner)")
    ap.add_argument("--path", default="auto", choices=("auto", "single", "team", "lds"),
                    help="growth path of a profiled plain leg (default: the library's choice)")
    ap.add_argument("--profile-leg", default=None,
                    choices=("plain2d", "plain3d", "batch2d", "batch3d", "copy", "stats"),
                    help="run only this leg (plain2d, plain3d, batch2d, batch3d, copy) for a "
                         "profiler, or the counting-build leg (stats, with WOLFF_LIBRARY=stats); "
                         "prints that leg's numbers instead of the benchmark line")
    return ap


def main():
    ap = build_parser()
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(independent lattices would shard across GPUs with no exchange).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1110_0899_amd import binding, workloads

    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.set_device(0)
    binding.load()
    legs = [s.strip() for s in args.legs.split(",") if s.strip()]
    extra = {"context": PAPER_CONTEXT}

    if args.profile_leg:
        profile_only(args, binding, workloads)
        return

    if "plain2d" not in legs:
        # studies only (no headline): the paper's size and temperature sweeps
        out = {}
        if "sizes" in legs:
            out["sizes"] = sizes_leg(binding, workloads, args.sweep_cpu_seconds)
        if "temps" in legs:
            out["temps"] = temps_leg(binding, workloads, args.sweep_cpu_seconds)
        if "potts" in legs:
            out["potts"] = potts_leg(binding, workloads, args)
        if "handoff" in legs:
            out["handoff"] = handoff_leg()
        print(json.dumps(out), flush=True)
        return

    main_leg = plain_leg(binding, 2, 4096, workloads.TC_2D, 2, max(args.warmup, MIN_THERM[2]),
                         args.steps)
    cpu = cpu_baseline(main_leg, args.cpu_seconds)
    if "plain3d" in legs:
        l3 = plain_leg(binding, 3, 256, workloads.T_3D, 3, max(3 * args.warmup, MIN_THERM[3]),
                       5 * args.steps)
        extra["plain_3d_L256"] = {k: v for k, v in l3.items()
                                  if k not in ("records", "checkpoint")}
    if "batch2d" in legs:
        extra["batch_2d_L4096"] = batch_leg(binding, workloads, 2, 4096, args.batch_replicas,
                                            args.batch_warmup, args.batch_steps)
        extra["batch_2d_L4096"]["vs_plain"] = (extra["batch_2d_L4096"]["added_per_s"]
                                               / main_leg["added_per_s"])
        c = counter_summary("batch_kernel", "batch_2d_L4096x%d" % args.batch_replicas)
        extra["batch_2d_L4096"]["traffic_bytes_per_added_spin"] = (
            None if c is None else c.get("hbm_bytes_per_added_spin"))
    if "batch3d" in legs:
        extra["batch_3d_L256"] = batch_leg(binding, workloads, 3, 256, args.batch_replicas,
                                           10 * args.batch_warmup, 5 * args.batch_steps)
        if "plain_3d_L256" in extra:
            extra["batch_3d_L256"]["vs_plain"] = (extra["batch_3d_L256"]["added_per_s"]
                                                  / extra["plain_3d_L256"]["added_per_s"])

    if "updateonly" in legs:
        # the paper's Table 1 reports both modes: "update only" and "+ measurement"
        u2 = plain_leg(binding, 2, 4096, workloads.TC_2D, 2, max(args.warmup, MIN_THERM[2]),
                       args.steps, measure=False)
        extra["plain_2d_L4096_update_only"] = {k: v for k, v in u2.items()
                                               if k not in ("records", "checkpoint")}
        if "plain3d" in legs:
            u3 = plain_leg(binding, 3, 256, workloads.T_3D, 3, max(3 * args.warmup, MIN_THERM[3]),
                           5 * args.steps, measure=False)
            extra["plain_3d_L256_update_only"] = {k: v for k, v in u3.items()
                                                  if k not in ("records", "checkpoint")}
    if "c1" in legs:
        extra["c1_2d_L32"] = c1_leg(binding, workloads)
    if "c4" in legs:
        extra["c4_mixed_batch"] = c4_leg(binding, workloads, args.c4_updates)
    if "serve" in legs:
        extra["serve_stream"] = serve_leg(binding, workloads)
    if "stats" in legs:
        extra["counting_build"] = stats_leg()
    copy_gbs = copy_peak_gbs()
    log("device copy: %.0f GB/s" % copy_gbs)
    for leg in extra.values():
        if isinstance(leg, dict) and "kernel_GBs_algorithmic" in leg:
            leg["kernel_frac_of_measured_copy"] = leg["kernel_GBs_algorithmic"] / copy_gbs

    achieved = main_leg["grow_GBs_algorithmic"]
    kernel, path_desc = {
        binding.PATH_TEAM: ("team_kernel", "multi-workgroup team kernel"),
        binding.PATH_LDS: ("lds_kernel", "LDS-resident lattice, 16 slabs of 256 rows, 512 threads each"),
        binding.PATH_SINGLE: ("batch_kernel", "one-workgroup kernel"),
    }[main_leg["path"]]
    # committed counters of that kernel at this workload, if taken on the current sources
    added_per_launch = main_leg["added"] / max(main_leg["grow_launches"], 1)
    traffic = counter_traffic(kernel, "2d_L4096", added_per_launch)
    out = {
        "metric": "added spins/s at Tc, 2D L=4096 & 3D L=256; % HBM peak; batched vs plain",
        "value": main_leg["added_per_s"],
        "unit": "added spins/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * main_leg["wall_s"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8 spins, u32 Philox draws, int64 sums",
        "data": "synthetic (seeded lattices; no dataset)",
        "config": {
            "workload": "2d_L4096_Tc_plain",
            "dim": 2, "L": 4096, "T": workloads.TC_2D, "J": 1.0, "seed": 2,
            "start": "ordered, thermalised at T_c before the timed updates",
            "thermalisation_updates": main_leg["warmup"],
            "mean_cluster_size_last_thermalisation": main_leg["therm_mean_csize"],
            "path": "plain one-lattice launch path (%s)" % path_desc,
            "measurement": "E and M after every update",
            "mean_cluster_size": main_leg["mean_csize"],
            "updates_per_s": main_leg["updates_per_s"],
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kernel + " (cluster growth)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "measured_copy_GBs": copy_gbs,
            "frac_of_measured_copy": achieved / copy_gbs,
            "bytes_per_added_spin": BYTES_PER_ADDED[2],
            "launches": main_leg["grow_launches"],
            "avg_launch_ms": main_leg["grow_ms"] / max(main_leg["grow_launches"], 1),
            "added_per_launch": added_per_launch,
            "traffic_bytes_per_added_spin": (None if traffic is None
                                             else traffic / max(added_per_launch, 1.0)),
        },
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
