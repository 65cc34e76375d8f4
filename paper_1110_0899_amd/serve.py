"""Serving driver: a real-time Poisson stream of Wolff jobs through the
library's continuous-batching request loop (wolff_server_*).

Jobs are submitted at their arrival times (wall clock); between quanta the
loop admits what fits (the C++ scheduler decides by slots and HBM
footprint), and every finished job's latency (arrival to records on the
host) is recorded.  All arithmetic runs in the library's HIP kernels.
"""
from __future__ import annotations

import time

import numpy as np

from . import binding


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else float("nan")


def run_stream(jobs, quantum_ms: float = 5.0, hbm_budget: int = 0, max_slots: int = 0,
               max_wall_s: float | None = None, keep_records: bool = False,
               update_only: bool = False, keep_finish_times: bool = False, progress=None):
    """Serve `jobs` (objects with dim, L, J, T, seed, n_updates, arrival_s).

    Returns a dict with per-job latency, p50/p99, aggregate added spins/s and
    the scheduler statistics.  With max_wall_s, arrivals stop at that time
    and the loop drains what was submitted."""
    order = sorted(range(len(jobs)), key=lambda k: jobs[k].arrival_s)
    srv = binding.Server(hbm_budget, max_slots)
    arrival, latency, records, index_of, finish = {}, {}, {}, {}, []
    added = 0
    t0 = time.perf_counter()
    i = 0
    submitted = 0
    max_queue = 0
    last_report = 0.0
    while True:
        now = time.perf_counter() - t0
        while i < len(order) and jobs[order[i]].arrival_s <= now and \
                (max_wall_s is None or jobs[order[i]].arrival_s <= max_wall_s):
            j = jobs[order[i]]
            jid = srv.submit(j, update_only=update_only)
            arrival[jid] = j.arrival_s
            index_of[jid] = order[i]
            submitted += 1
            i += 1
        st = srv.stats()
        max_queue = max(max_queue, st["queued"])
        arrivals_over = i >= len(order) or (max_wall_s is not None
                                            and jobs[order[i]].arrival_s > max_wall_s)
        if st["queued"] == 0 and st["running"] == 0:
            if arrivals_over:
                break
            # idle: wait for the next arrival
            time.sleep(max(0.0, min(jobs[order[i]].arrival_s - now, 0.01)))
            continue
        srv.step(quantum_ms)
        done_t = time.perf_counter() - t0
        if progress is not None and done_t - last_report > 5.0:
            last_report = done_t
            progress("serve t=%.1f s: submitted %d, finished %d, queued %d, running %d"
                     % (done_t, submitted, len(latency), st["queued"], st["running"]))
        for jid in srv.finished():
            rec = srv.take(jid)
            latency[jid] = done_t - arrival[jid]
            finish.append(done_t)
            added += int(rec["csize"].sum())
            if keep_records:
                records[index_of[jid]] = rec
    wall = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    lat = list(latency.values())
    return {
        "jobs": len(lat), "wall_s": wall,
        "p50_latency_s": percentile(lat, 50), "p99_latency_s": percentile(lat, 99),
        "mean_latency_s": float(np.mean(lat)) if lat else float("nan"),
        "added_spins": added, "added_per_s": added / wall if wall > 0 else 0.0,
        "jobs_per_s": len(lat) / wall if wall > 0 else 0.0,
        "max_queue_depth": max_queue, "quanta": stats["quanta"],
        "gpu_ms": stats["gpu_ms"], "slots": stats["slots"],
        "budget_bytes": stats["budget_bytes"],
        "records": records,
        "finish_s": finish if keep_finish_times else None,
    }


def capacity(jobs, quantum_ms: float = 5.0, hbm_budget: int = 0, update_only: bool = False,
             progress=None) -> dict:
    """Saturated throughput of the loop, measured.

    Every job of `jobs` (more than the loop's slots) is queued at time 0, so
    the loop runs full until the queue empties; the capacity is the rate of
    completions between the first and the last fifth of them (the start-up
    ramp and the drain tail excluded)."""
    closed = [type(j)(**{**j.as_dict(), "arrival_s": 0.0}) for j in jobs]
    r = run_stream(closed, quantum_ms=quantum_ms, hbm_budget=hbm_budget, update_only=update_only,
                   keep_finish_times=True, progress=progress)
    fin = np.sort(np.asarray(r["finish_s"], dtype=np.float64))
    n = len(fin)
    lo, hi = n // 5, (4 * n) // 5
    rate = (hi - lo) / (fin[hi] - fin[lo]) if hi > lo and fin[hi] > fin[lo] else n / r["wall_s"]
    return {"jobs_per_s": float(rate), "jobs": n, "slots": r["slots"],
            "closed_batch_wall_s": r["wall_s"], "closed_batch_jobs_per_s": n / r["wall_s"],
            "closed_batch_added_per_s": r["added_per_s"],
            "window": "completions %d..%d of %d" % (lo, hi, n)}
