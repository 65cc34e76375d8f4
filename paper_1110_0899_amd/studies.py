"""Binder-ratio scan through the batched form (Section 5, Fig. 2):

    U(T) = 1 - <M^4> / (3 <M^2>^2)

for several lattice sizes over a temperature grid; the curves of different
L cross near T_c.  Every (L, T) point is one replica of one persistent
batched launch; the magnetisation series comes from the per-update records.

    python -m paper_1110_0899_amd.studies binder --dim 2 --L 8,16,32,64 \\
        --T 2.20,2.24,2.269185,2.30,2.34 --discard 5000 --measure 50000 [--out scan.json]

The paper discards 5000 and measures 50000 updates in 2D (10000 and 100000
in 3D) at L = 512..4096 (64..256 in 3D); at those sizes one replica per
workgroup needs hours, so the scan is run at smaller L, where the crossing
is already resolved.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import binding, workloads


def binder_ratio(M) -> float:
    """U = 1 - <M^4> / (3 <M^2>^2) of a magnetisation series."""
    m = np.asarray(M, dtype=np.float64)
    m2 = np.mean(m * m)
    m4 = np.mean(m ** 4)
    return float(1.0 - m4 / (3.0 * m2 * m2))


def binder_error(M, nblocks: int = 20) -> float:
    """Jackknife error of U over contiguous blocks of a correlated series."""
    m = np.asarray(M, dtype=np.float64)
    n = (len(m) // nblocks) * nblocks
    if n == 0:
        return float("nan")
    blocks = m[:n].reshape(nblocks, -1)
    s2 = (blocks ** 2).sum(axis=1)
    s4 = (blocks ** 4).sum(axis=1)
    per = blocks.shape[1]
    tot2, tot4 = s2.sum(), s4.sum()
    jack = []
    for b in range(nblocks):
        c = n - per
        m2 = (tot2 - s2[b]) / c
        m4 = (tot4 - s4[b]) / c
        jack.append(1.0 - m4 / (3.0 * m2 * m2))
    jack = np.asarray(jack)
    return float(math.sqrt((nblocks - 1) * np.mean((jack - jack.mean()) ** 2)))


def binder_scan(dim: int, Ls, Ts, discard: int, measure: int, seed0: int = 0x42000000,
                start: int = 1, log=None) -> list[dict]:
    """One batched launch over every (L, T); returns one row per point with
    U, its error, <|M|>/N, <|C|>/N and the mean bond sum per site."""
    jobs, keys = [], []
    for L in Ls:
        for T in Ts:
            jobs.append(workloads.Job(dim, int(L), float(T), seed0 + len(jobs), discard + measure))
            keys.append((int(L), float(T)))
    t0 = time.time()
    rows = []
    with binding.Batch(jobs, start=start) as b:
        b.set_measure(True)
        b.run()
        for i, (L, T) in enumerate(keys):
            rec = b.records(i)
            N = L ** dim
            M = rec["mag"][discard:].astype(np.float64)
            C = rec["csize"][discard:].astype(np.float64)
            Bs = rec["bond_sum"][discard:].astype(np.float64)
            rows.append({"dim": dim, "L": L, "T": T, "updates": measure, "discarded": discard,
                         "U": binder_ratio(M), "U_err": binder_error(M),
                         "abs_m": float(np.mean(np.abs(M)) / N), "csize_frac": float(np.mean(C) / N),
                         "bond_per_site": float(np.mean(Bs) / N)})
    if log:
        log("binder scan %dD, L=%s, %d temperatures, %d+%d updates: %.1f s"
            % (dim, ",".join(str(L) for L in Ls), len(Ts), discard, measure, time.time() - t0))
    return rows


def crossing(rows, L1: int, L2: int):
    """Temperature where U(L1) and U(L2) cross, by linear interpolation
    between the grid points that bracket the sign change (None if none)."""
    a = sorted((r["T"], r["U"]) for r in rows if r["L"] == L1)
    b = dict((r["T"], r["U"]) for r in rows if r["L"] == L2)
    prev = None
    for T, u1 in a:
        if T not in b:
            continue
        d = u1 - b[T]
        if prev is not None and (prev[1] > 0) != (d > 0):
            T0, d0 = prev
            return T0 + (T - T0) * d0 / (d0 - d)
        prev = (T, d)
    return None


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("binder")
    s.add_argument("--dim", type=int, default=2)
    s.add_argument("--L", default="8,16,32,64")
    s.add_argument("--T", default=None, help="comma-separated temperatures (default: around T_c)")
    s.add_argument("--discard", type=int, default=5000)
    s.add_argument("--measure", type=int, default=50000)
    s.add_argument("--out", default=None)
    a = ap.parse_args()
    binding.load()
    Ls = [int(v) for v in a.L.split(",")]
    if a.T:
        Ts = [float(v) for v in a.T.split(",")]
    else:
        Tc = workloads.TC_2D if a.dim == 2 else workloads.T_3D
        Ts = [Tc * f for f in (0.97, 0.985, 1.0, 1.015, 1.03)]
    rows = binder_scan(a.dim, Ls, Ts, a.discard, a.measure,
                       log=lambda m: print("[studies] " + m, flush=True))
    out = {"rows": rows, "crossings": {"%d/%d" % (Ls[i], Ls[i + 1]): crossing(rows, Ls[i], Ls[i + 1])
                                       for i in range(len(Ls) - 1)}}
    for r in rows:
        print("L=%4d T=%.6f U=%.5f +- %.5f |m|=%.4f" % (r["L"], r["T"], r["U"], r["U_err"], r["abs_m"]))
    print(json.dumps(out["crossings"]))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
