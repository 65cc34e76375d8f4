"""Pins of the oracle's q-state Potts extension (Section 6): the q = 2 case
against the Ising oracle, exact enumeration for q = 3 and 4, the cluster as a
connected component, the new-colour draw, and the limiting temperatures."""
import numpy as np
import pytest

import exact_ising
import exact_potts
import oracle

TC2 = 2.0 / np.log(1.0 + np.sqrt(2.0))


def potts_pin_ising_equivalence(o):
    # q = 2 with J_Potts = 2 is the Ising update with J = 1: same threshold,
    # colour 0 <-> +1, and the records coincide exactly
    for dim, L, T, seed, n in [(2, 8, TC2, 3, 300), (2, 5, 2.5, 4, 200), (3, 4, 4.5, 5, 200),
                               (2, 2, 1.5, 6, 100), (3, 2, 3.0, 7, 100)]:
        assert o.potts_threshold(2.0, T) == o.threshold(1.0, T)
        C = o.potts_init(dim, L, 2, seed)
        S = o.init_spins(dim, L, seed)
        assert (S == 1 - 2 * C.astype(np.int16)).all()
        thr = o.threshold(1.0, T)
        ri = o.run(dim, L, thr, seed, 0, n, S)
        rp = o.potts_run(dim, L, 2, thr, seed, 0, n, C)
        assert (ri == rp).all(), (dim, L)
        assert (S == 1 - 2 * C.astype(np.int16)).all()


def potts_pin_enumeration(o):
    # stationarity: long runs reproduce the exact <B> and <M^2>
    for dim, L, q, T, seed in [(2, 3, 3, 1.0, 11), (3, 2, 3, 1.3, 12), (2, 3, 4, 0.9, 13)]:
        ex = exact_potts.exact_moments(dim, L, q, 1.0 / T)
        thr = o.potts_threshold(1.0, T)
        C = o.potts_init(dim, L, q, seed)
        rec = o.potts_run(dim, L, q, thr, seed, 0, 200_000, C)[2000:]
        mB, eB = exact_ising.block_mean_err(rec[:, 0])
        mM2, eM2 = exact_ising.block_mean_err(rec[:, 1].astype(np.float64) ** 2)
        assert abs(mB - ex["B"]) < 5 * eB + 1e-9, (dim, L, q, mB, ex["B"], eB)
        assert abs(mM2 - ex["M2"]) < 5 * eM2 + 1e-9, (dim, L, q, mM2, ex["M2"], eM2)


def potts_pin_cluster_is_component(o):
    rng = np.random.default_rng(21)
    for dim, L, q in [(2, 7, 3), (3, 4, 5), (2, 6, 4)]:
        C = rng.integers(0, q, size=L ** dim).astype(np.int8)
        thr = o.potts_threshold(1.0, 0.8)
        for t in range(5):
            member, s, s0 = o.cluster(dim, L, thr, 31, t, C)
            assert s0 == C[s]
            labels = exact_ising.active_bond_components(
                dim, L, C, lambda b, mu: o.bond_draw(31, t, s, b, mu) < thr)
            assert (member.astype(bool) == (labels == labels[s])).all()


def potts_pin_new_colour(o):
    # never the old colour; uniform over the q - 1 others
    q = 5
    counts = np.zeros((q, q), dtype=np.int64)
    for t in range(40_000):
        s0 = t % q
        c = o.potts_new_colour(77, t, q, s0)
        assert 0 <= c < q and c != s0
        counts[s0, c] += 1
    for s0 in range(q):
        row = np.delete(counts[s0], s0)
        exp = row.sum() / (q - 1)
        chi2 = ((row - exp) ** 2 / exp).sum()
        assert chi2 < 20.0, (s0, row)          # 3 degrees of freedom


def potts_pin_special_cases(o):
    dim, L, q, N = 2, 6, 4, 36
    # T -> infinity: thr = 0, single-site clusters; M moves by q or 0
    C = o.potts_init(dim, L, q, 9)
    rec = o.potts_run(dim, L, q, 0, 9, 0, 50, C)
    assert (rec[:, 2] == 1).all()
    assert set(np.abs(np.diff(rec[:, 1]))) <= {0, q}
    # T -> 0 from one colour: the cluster is the whole lattice each update
    C = np.zeros(N, dtype=np.int8)
    thr = o.potts_threshold(1.0, 1e-3)
    rec = o.potts_run(dim, L, q, thr, 9, 0, 20, C)
    assert (rec[:, 2] == N).all() and (rec[:, 0] == 2 * N * (q - 1)).all()
    assert len(set(C.tolist())) == 1


ALL_POTTS_PINS = {
    "ising_equivalence": potts_pin_ising_equivalence,
    "special_cases": potts_pin_special_cases,
    "new_colour": potts_pin_new_colour,
    "cluster_is_component": potts_pin_cluster_is_component,
    "enumeration": potts_pin_enumeration,
}


@pytest.mark.parametrize("name", list(ALL_POTTS_PINS))
def test_potts_pin(name):
    ALL_POTTS_PINS[name](oracle.default())


MUTANTS = [
    ("potts_p_with_factor_2", "const double p = 1.0 - exp(-J / T);", "const double p = 1.0 - exp(-2.0 * J / T);"),
    ("potts_new_colour_may_stay", "return (s0 + 1 + r) % q;", "return (s0 + r) % q;"),
    ("potts_new_colour_biased", "(uint64_t)(q - 1)) >> 32", "(uint64_t)(q - 2)) >> 32"),
    ("potts_init_wrong_scale", "(uint64_t)q) >> 32);", "(uint64_t)(q - 1)) >> 32);"),
    ("potts_magnetisation_count", "m += (S[i] == 0) ? q - 1 : -1;", "m += (S[i] == 0) ? 1 : 0;"),
    ("potts_bond_sum_count", "b += (S[i] == S[k]) ? q - 1 : -1;", "b += (S[i] == S[k]) ? 1 : 0;"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_potts_mutant_is_rejected(tmp_path, name, old, new):
    src = open(oracle.SOURCE).read()
    assert old in src, name
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = oracle.compile_oracle(str(path), str(tmp_path / "libmutant.so"))
    o = oracle.Oracle(lib)
    for pin in ALL_POTTS_PINS.values():
        try:
            pin(o)
        except (AssertionError, RuntimeError):
            return
    pytest.fail("mutant %s passed every Potts pin" % name)
