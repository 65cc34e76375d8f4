"""Pins for the CPU oracle: checks against what the paper and the mathematics
fix, never against the oracle's own formulas retyped.

Each check takes an ``oracle.Oracle`` instance and raises AssertionError when
it fails, so the same checks run on the real oracle (tests/test_oracle.py)
and on deliberately broken copies of it (tests/test_oracle_mutants.py).
"""
from __future__ import annotations

import math
import os
import subprocess

import mpmath as mp
import numpy as np

import exact_ising as ex

HERE = os.path.dirname(os.path.abspath(__file__))
XCHECK_SRC = os.path.join(HERE, "xcheck", "rocrand_philox_ref.cpp")
XCHECK_BIN = os.path.join(HERE, "xcheck", "rocrand_philox_ref")

# Critical temperature of the square lattice, T_c/J = 2/ln(1+sqrt 2) = 2.269...
# (Section 1 and Section 5 quote 2.269); the simple-cubic value used by the
# workloads is 4.511528 (Section 5 quotes 4.510).
TC_2D = 2.0 / math.log(1.0 + math.sqrt(2.0))
T_3D = 4.511528


# ------------------------------------------------------------------ Philox
def build_rocrand_reference() -> str | None:
    """Build the rocRAND-backed Philox reference program (host code)."""
    if os.path.exists(XCHECK_BIN) and os.path.getmtime(XCHECK_BIN) >= os.path.getmtime(XCHECK_SRC):
        return XCHECK_BIN
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        return None
    tmp = XCHECK_BIN + ".tmp%d" % os.getpid()
    subprocess.check_call([hipcc, "-O1", "-o", tmp, XCHECK_SRC],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    os.replace(tmp, XCHECK_BIN)
    return XCHECK_BIN


def rocrand_blocks(requests: np.ndarray) -> np.ndarray:
    """requests: uint32 [n, 6] = key0 key1 c0 c1 c2 c3 -> uint32 [n, 4] from rocRAND."""
    exe = build_rocrand_reference()
    assert exe is not None, "hipcc not available to build the rocRAND reference"
    text = "\n".join(" ".join(str(int(v)) for v in row) for row in requests) + "\n"
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()],
                    dtype=np.uint64).astype(np.uint32)


def pin_philox_vs_rocrand(orc, n: int = 3000, seed: int = 12345):
    rng = np.random.default_rng(seed)
    req = rng.integers(0, 2 ** 32, size=(n, 6), dtype=np.uint64)
    req[:, 3] &= (1 << 30) - 1          # the reference maps (c1:c0) to an element offset * 4
    # structured cases: zero key / counter, all-ones words, the counters the method uses
    req[0] = [0, 0, 0, 0, 0, 0]
    req[1] = [0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, (1 << 30) - 1, 0xFFFFFFFF, 0xFFFFFFFF]
    req[2] = [1, 0, 17, 5, 3, 0]        # bond draw: (b, t, s, 0)
    req[3] = [1, 0, 0, 9, 0, 1]         # seed-site draw: (0, t, 0, 1)
    req[4] = [1, 0, 33, 0, 0, 2]        # initial spin: (i, 0, 0, 2)
    ref = rocrand_blocks(req)
    mine = np.array([orc.philox(r[2:6], r[0:2]) for r in req], dtype=np.uint32)
    bad = np.nonzero((mine != ref).any(axis=1))[0]
    assert bad.size == 0, "Philox differs from rocRAND at %d requests, first %s: %s vs %s" % (
        bad.size, req[bad[0]].tolist(), mine[bad[0]].tolist(), ref[bad[0]].tolist())


# --------------------------------------------------------------- threshold
def exact_threshold(J, T) -> int:
    """floor((1 - exp(-2J/T)) 2^32) evaluated with 50 significant digits."""
    with mp.workdps(50):
        p = 1 - mp.exp(-2 * mp.mpf(J) / mp.mpf(T))
        v = mp.floor(p * mp.mpf(2) ** 32)
        frac = p * mp.mpf(2) ** 32 - v
        return int(v), float(frac)


def pin_threshold(orc):
    # Closed form at the 2D critical point: exp(-2K_c) = sqrt2 - 1, so p = 2 - sqrt 2.
    with mp.workdps(50):
        thr_c = int(mp.floor((2 - mp.sqrt(2)) * mp.mpf(2) ** 32))
    assert orc.threshold(1.0, TC_2D) == thr_c, (orc.threshold(1.0, TC_2D), thr_c)
    for J, T in [(1.0, T_3D), (1.0, 2.0), (1.0, 2.6), (1.0, 4.3), (1.0, 4.7), (0.5, 1.1),
                 (2.0, 7.0), (1.0, 0.9)]:
        v, frac = exact_threshold(J, T)
        assert 1e-6 < frac < 1 - 1e-6, "threshold too close to an integer for a binary64 check"
        assert orc.threshold(J, T) == v, (J, T, orc.threshold(J, T), v)
    # limits: T -> infinity gives p -> 0; T -> 0 gives p -> 1 (clamped to 2^32 - 1)
    assert orc.threshold(1.0, 1e300) == 0
    assert orc.threshold(1.0, 1e-300) == 0xFFFFFFFF


# --------------------------------------------------------------- seed site
def pin_seed_site(orc):
    rng = np.random.default_rng(7)
    # range and uniformity on a non-power-of-two N (chi-square, 63 dof)
    N, n = 63, 63 * 400
    counts = np.zeros(N, dtype=np.int64)
    for t in range(n):
        s = orc.seed_site(3, t, N)
        assert 0 <= s < N
        counts[s] += 1
    chi2 = float(((counts - n / N) ** 2 / (n / N)).sum())
    assert chi2 < 130.0, chi2            # P(chi2_62 > 130) ~ 1e-6
    # N = 2^k: the multiply-high is exactly the top k bits of the 64-bit draw,
    # and the top k bits of a uniform draw are uniform; compare with rocRAND's
    # independently generated words.
    ts = rng.integers(0, 2 ** 30, size=40)
    blks = rocrand_blocks(np.array([[3, 0, 0, int(t), 0, 1] for t in ts], dtype=np.uint64))
    for k in (1, 5, 12, 24, 32):
        N = 1 << k
        for t, blk in zip(ts, blks):
            u = (int(blk[1]) << 32) | int(blk[0])
            assert orc.seed_site(3, int(t), N) == u >> (64 - k)
    # N = 1: only site 0 exists
    assert orc.seed_site(9, 5, 1) == 0


# ---------------------------------------------------------- initial state
def pin_init_spins(orc):
    S = orc.init_spins(2, 256, 11)
    assert set(np.unique(S).tolist()) <= {-1, 1}
    n = S.size
    m = float(S.astype(np.int64).sum())
    assert abs(m) < 5 * math.sqrt(n), m               # P(+1) = 1/2
    nb = ex.neighbour_tables(2, 256)[0]
    c = float((S.astype(np.int64) * S[nb]).sum())
    assert abs(c) < 5 * math.sqrt(n), c               # independent sites
    # the initial spin uses word 0 of the domain-2 block (rocRAND reference)
    idx = np.array([0, 1, 2, 255, 256, 40000, 65535])
    req = np.array([[11, 0, int(i), 0, 0, 2] for i in idx], dtype=np.uint64)
    words = rocrand_blocks(req)[:, 0]
    expect = np.where(words < 2 ** 31, 1, -1)
    assert (S[idx] == expect).all()


# ------------------------------------------------------ cluster = component
def pin_cluster_is_component(orc, cases=None):
    """The oracle's cluster equals the connected component of the seed site in
    the graph of active bonds between spins equal to s0, with every bond
    drawn once from its own key and compared with the threshold."""
    if cases is None:
        cases = [(2, 2, 2.0), (2, 3, TC_2D), (2, 5, 1.5), (2, 16, TC_2D), (2, 33, 2.6),
                 (3, 2, 4.0), (3, 3, T_3D), (3, 8, T_3D), (3, 7, 3.5)]
    for dim, L, T in cases:
        thr = orc.threshold(1.0, T)
        seed = 1000 + 7 * L + dim
        S = orc.init_spins(dim, L, seed)
        orc.run(dim, L, thr, seed, 0, 5, S)           # move away from the start
        for t in range(5, 11):
            member, s, s0 = orc.cluster(dim, L, thr, seed, t, S)
            assert S[s] == s0
            def active(b, mu, t=t, s=s):
                return orc.bond_draw(seed, t, s, b, mu) < thr

            labels = ex.active_bond_components(dim, L, S, active)
            expect = ((labels == labels[s]) & (S == s0)).astype(np.uint8)
            assert (member == expect).all(), (dim, L, T, t, int(member.sum()), int(expect.sum()))
            # same cluster, flipped, is what run() applies
            S2 = S.copy()
            rec = orc.run(dim, L, thr, seed, t, 1, S2)
            assert int(rec[0, 2]) == int(member.sum())
            assert (S2 == np.where(member == 1, -S, S)).all()
            S[:] = S2


# ------------------------------------------------ stationarity (enumeration)
def pin_enumeration(orc, cases=None, n_updates=300_000, zmax=4.5):
    """Long-run averages of the oracle's chain against exact Boltzmann averages
    of the enumerated lattice, and the improved estimator <|C|> = <M^2>/N."""
    if cases is None:
        cases = [(2, 4, TC_2D), (2, 4, 1.6), (2, 4, 4.0), (2, 3, 2.0),
                 (3, 2, T_3D), (3, 2, 2.5), (2, 2, 3.0)]
    for dim, L, T in cases:
        K = 1.0 / T
        exact = ex.exact_moments(dim, L, K)
        N = exact["N"]
        thr = orc.threshold(1.0, T)
        seed = 77 + L * 10 + dim
        S = orc.init_spins(dim, L, seed)
        orc.run(dim, L, thr, seed, 0, 1000, S)
        rec = orc.run(dim, L, thr, seed, 1000, n_updates, S)
        B = rec[:, 0].astype(np.float64)
        M = rec[:, 1].astype(np.float64)
        C = rec[:, 2].astype(np.float64)
        checks = {
            "B": (B, exact["B"]),
            "M2": (M ** 2, exact["M2"]),
            "absM": (np.abs(M), exact["absM"]),
            "M4": (M ** 4, exact["M4"]),
            "C": (C, exact["M2"] / N),            # improved estimator <|C|> = <M^2>/N
        }
        for name, (series, target) in checks.items():
            mean, err = ex.block_mean_err(series)
            z = (mean - target) / max(err, 1e-12)
            assert abs(z) < zmax, (dim, L, T, name, mean, target, err, z)
        # joint (B, M) histogram: total-variation distance to the exact law
        keys = exact["key_of"](rec[:, 0], rec[:, 1])
        uniq, cnt = np.unique(keys, return_counts=True)
        emp = dict(zip(uniq.tolist(), (cnt / len(keys)).tolist()))
        tv = 0.5 * sum(abs(emp.get(k, 0.0) - p) for k, p in
                       zip(exact["dist_keys"].tolist(), exact["dist_prob"].tolist()))
        tv += 0.5 * sum(v for k, v in emp.items() if k not in set(exact["dist_keys"].tolist()))
        assert tv < 0.01, (dim, L, T, tv)


# ----------------------------------------- exact 2D energy (Kaufman / F-F)
def pin_exact_energy_2d(orc, L=32, n_therm=1000, n_meas=30_000, seed=1, zmax=4.5):
    thr = orc.threshold(1.0, TC_2D)
    S = orc.init_spins(2, L, seed)
    orc.run(2, L, thr, seed, 0, n_therm, S)
    rec = orc.run(2, L, thr, seed, n_therm, n_meas, S)
    N = L * L
    mean, err = ex.block_mean_err(rec[:, 0] / N)
    exact = ex.kaufman_mean_B(L, 1.0 / TC_2D) / N
    z = (mean - exact) / err
    assert abs(z) < zmax, (mean, exact, err, z)
    # improved estimator inside the same run
    cm, ce = ex.block_mean_err(rec[:, 2].astype(np.float64))
    mm, me = ex.block_mean_err(rec[:, 1].astype(np.float64) ** 2 / N)
    z2 = (cm - mm) / math.hypot(ce, me)
    assert abs(z2) < zmax, (cm, mm, ce, me)
    return mean, err, exact


# --------------------------------------------------------- special cases
def pin_special_cases(orc):
    for dim, L in [(2, 8), (3, 4), (2, 5)]:
        N = L ** dim
        # T -> infinity: p = 0, no bond is ever active: |C| = 1 and |dM| = 2
        thr = orc.threshold(1.0, 1e300)
        assert thr == 0
        S = orc.init_spins(dim, L, 5)
        _, M0 = orc.observables(dim, L, S)
        rec = orc.run(dim, L, thr, 5, 0, 200, S)
        assert (rec[:, 2] == 1).all()
        dM = np.diff(np.concatenate([[M0], rec[:, 1]]))
        assert (np.abs(dM) == 2).all()
        # T -> 0 from the all-up state: every bond active, the cluster is the lattice
        thr = orc.threshold(1.0, 1e-3)
        S = np.ones(N, dtype=np.int8)
        rec = orc.run(dim, L, thr, 6, 0, 20, S)
        assert (rec[:, 2] == N).all()
        assert (np.abs(rec[:, 1]) == N).all()
        assert (rec[:, 0] == dim * N).all()          # all bonds satisfied: B = dN


# ------------------------------------------------------------- invariants
def pin_invariants(orc):
    for dim, L, T in [(2, 32, TC_2D), (3, 6, T_3D), (2, 7, 2.2)]:
        thr = orc.threshold(1.0, T)
        S = orc.init_spins(dim, L, 21)
        B0, M0 = orc.observables(dim, L, S)
        assert B0 == ex.bond_sum(dim, L, S) and M0 == int(S.astype(np.int64).sum())
        A = S.copy()
        ra = orc.run(dim, L, thr, 21, 0, 300, A)
        Bx = S.copy()
        r1 = orc.run(dim, L, thr, 21, 0, 120, Bx)
        r2 = orc.run(dim, L, thr, 21, 120, 180, Bx)
        assert (A == Bx).all()
        assert (ra == np.concatenate([r1, r2])).all()
        # recorded observables agree with an independent recount of the final state
        assert ra[-1, 0] == ex.bond_sum(dim, L, A)
        assert ra[-1, 1] == int(A.astype(np.int64).sum())


ALL_PINS = {
    "philox_vs_rocrand": pin_philox_vs_rocrand,
    "threshold": pin_threshold,
    "seed_site": pin_seed_site,
    "init_spins": pin_init_spins,
    "cluster_is_component": pin_cluster_is_component,
    "enumeration": pin_enumeration,
    "exact_energy_2d": pin_exact_energy_2d,
    "special_cases": pin_special_cases,
    "invariants": pin_invariants,
}
