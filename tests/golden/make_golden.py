"""Writes tests/golden/c1_oracle.txt from the CPU oracle only.

Workload: square lattice L = 32, periodic, J = 1, T = 2/ln(1+sqrt 2) (the
critical temperature of Section 5), seed 1, updates 0 .. 9999 from the iid
+-1 start.  Records (B, M, |C|) after each update, E = -J B (Section 5's
"+ measurement"; Wolff steps (i)-(v) of Section 2).

The fixture freezes the oracle's output so that any later change to its
arithmetic shows up as a failing test and has to be justified.
Run:  python tests/golden/make_golden.py
"""
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402

TC_2D = 2.0 / np.log(1.0 + np.sqrt(2.0))


def main():
    dim, L, seed, n = 2, 32, 1, 10_000
    thr = oracle.threshold(1.0, TC_2D)
    S = oracle.init_spins(dim, L, seed)
    h0 = hashlib.sha256(S.tobytes()).hexdigest()
    rec = oracle.run(dim, L, thr, seed, 0, n, S)
    h1 = hashlib.sha256(S.tobytes()).hexdigest()
    out = os.path.join(HERE, "c1_oracle.txt")
    with open(out, "w") as f:
        f.write("# CPU oracle, square lattice L=32, T=2/ln(1+sqrt2), J=1, seed=1, 10000 updates\n")
        f.write("# written by tests/golden/make_golden.py (oracle only)\n")
        f.write("threshold %d\n" % thr)
        f.write("init_spins_sha256 %s\n" % h0)
        f.write("final_spins_sha256 %s\n" % h1)
        f.write("sum_csize %d\n" % int(rec[:, 2].sum()))
        f.write("sum_B %d\n" % int(rec[:, 0].sum()))
        f.write("sum_M %d\n" % int(rec[:, 1].sum()))
        f.write("# first 200 records: t B M csize\n")
        for t in range(200):
            f.write("%d %d %d %d\n" % (t, rec[t, 0], rec[t, 1], rec[t, 2]))


if __name__ == "__main__":
    main()
