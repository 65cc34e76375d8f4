"""Autotuner for the batched kernel's tile sizes (workgroup size, LDS frontier
ring entries).

Every candidate runs the *same* replicas from the same state for the same
updates (the random stream does not depend on the tiles, so the work is
identical and the results bit-equal), and the candidate with the shortest
kernel time wins.  Results are cached in a JSON file keyed by
(GPU architecture, dim, log2 of L rounded up, replica count class); the file
is $WOLFF_TUNE_CACHE or ~/.cache/wolff_mi355x_tune.json (Potts replica sets
have keys of their own, and so does each mixed set of shapes).
"""
from __future__ import annotations

import json
import math
import os
import time

from . import binding

# (1024, 4096) is left out: in the tuner's short runs from the ordered start
# it can look best for 3D L=256 while it is ~20 % slower than (512, 2048)
# over a thermalised window on MI355X.
CANDIDATES = [(128, 2048), (256, 2048), (256, 4096), (512, 2048), (512, 4096)]


def cache_path() -> str:
    return os.environ.get("WOLFF_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "wolff_mi355x_tune.json"))


def _arch() -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def key(dim: int, L: int, n_replicas: int, q: int = 0) -> str:
    k = "%s|d%d|L2^%d|B2^%d" % (_arch(), dim, math.ceil(math.log2(max(L, 2))),
                                math.ceil(math.log2(max(n_replicas, 1))))
    return k + ("|potts" if q else "")


def _load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(k: str, v: dict):
    c = _load_cache()
    c[k] = v
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def measure(jobs, wg: int, q: int, warm: int, timed: int, start: int, lds: bool = True) -> float:
    """Kernel milliseconds of `timed` updates of every replica after `warm`
    (lds: the replicas that fit one workgroup's LDS on the LDS path, whose
    timing the tiles do not change)."""
    with binding.Batch(jobs, start=start) as b:
        b.set_lds(lds)
        b.set_tiles(wg, q)
        if warm:
            b.run(warm)
            b.last_ms()
        b.run(timed)
        return b.last_ms()


def set_key(jobs) -> str:
    """Cache key of a job list: the class of its jobs when they share one;
    else the class of its largest shape marked as mixed, with a digest of
    every job's (dim, L, q), so that a mixed set never reads a same-class
    entry.  The key does not depend on the order of the jobs."""
    shapes = sorted((j.dim, j.L, getattr(j, "q", 0)) for j in jobs)
    classes = {key(d, L, len(jobs), q) for d, L, q in shapes}
    d, L, q = shapes[-1]
    k = key(d, L, len(jobs), q)
    if len(classes) > 1:
        import hashlib
        k += "|mixed:" + hashlib.sha256(repr(shapes).encode()).hexdigest()[:12]
    return k


def tune(jobs, warm: int = 4, timed: int = 4, start: int = 1, candidates=None,
         use_cache: bool = True, log=None, lds: bool = True) -> dict:
    """Best (wg, queue_entries) of the one-workgroup kernel for a list of
    jobs (cached per set_key and LDS setting)."""
    k = set_key(jobs) + ("" if lds else "|no-lds")
    if use_cache:
        hit = _load_cache().get(k)
        if hit:
            return hit
    cands = candidates or CANDIDATES
    best = None
    trials = []
    t0 = time.time()
    for wg, q in cands:
        ms = measure(jobs, wg, q, warm, timed, start, lds)
        trials.append({"wg": wg, "queue_entries": q, "ms": ms})
        if log:
            log("tune %s: wg=%d q=%d -> %.1f ms" % (k, wg, q, ms))
        if best is None or ms < best["ms"]:
            best = {"wg": wg, "queue_entries": q, "ms": ms}
    result = {"wg": best["wg"], "queue_entries": best["queue_entries"], "key": k,
              "trials": trials, "tune_seconds": time.time() - t0}
    _store(k, result)
    return result
