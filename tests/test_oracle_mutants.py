"""Planted mistakes: each copy of the oracle below carries one plausible bug
(a dropped term, a wrong index, a wrong constant, a wrong sign) and must be
rejected by at least one pin.  The mistakes are planted in temporary copies
of the oracle source, on the CPU; the real oracle is untouched."""
import os
import shutil

import pytest

import oracle
import pins

# (name, original text, replacement) applied to oracle/wolff_oracle.c
MUTANTS = [
    ("bond_base_always_j", "const uint64_t b = (sgn > 0) ? j : k;", "const uint64_t b = j;"),
    ("p_without_factor_2", "exp(-2.0 * J / T)", "exp(-J / T)"),
    ("threshold_rounded", "return (uint32_t)floor(scaled);", "return (uint32_t)floor(scaled + 0.5);"),
    ("philox_multiplier", "(uint64_t)0xD2511F53u", "(uint64_t)0xD2511F55u"),
    ("philox_key_bump", "k[1] += 0xBB67AE85u;", "k[1] += 0xBB67AE84u;"),
    ("philox_nine_rounds", "round < 10", "round < 9"),
    ("seed_site_range", "x[0])) * N;", "x[0])) * (N - 1);"),
    ("index_transposed", "for (int a = dim - 1; a >= 0; --a)", "for (int a = 0; a < dim; ++a)"),
    ("site0_never_flipped", "for (uint64_t i = 0; i < N; ++i)\n            if (member[i])",
     "for (uint64_t i = 1; i < N; ++i)\n            if (member[i])"),
    ("seed_spin_fixed", "const int8_t s0 = S[s];", "const int8_t s0 = 1;"),
    ("init_wrong_word", "S[i] = (x[0] < 0x80000000u)", "S[i] = (x[1] < 0x80000000u)"),
    ("bond_counter_without_t", "uint32_t ctr[4] = {(uint32_t)b, t, (uint32_t)s, 0u}, r[4];\n                orc",
     "uint32_t ctr[4] = {(uint32_t)b, 0u, (uint32_t)s, 0u}, r[4];\n                orc"),
    ("bond_word_fixed", "if (r[mu] < thr)", "if (r[0] < thr)"),
    ("energy_drops_last_axis", "for (int mu = 0; mu < dim; ++mu)\n            b +=",
     "for (int mu = 0; mu + 1 < dim; ++mu)\n            b +="),
]

# cheap pins first; a mutant is rejected at its first failing pin
ORDER = ["threshold", "philox_vs_rocrand", "special_cases", "invariants", "init_spins",
         "cluster_is_component", "seed_site", "enumeration", "exact_energy_2d"]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_rejected(tmp_path, name, old, new):
    src = open(oracle.SOURCE).read()
    assert src.count(old) == 1, "mutation anchor not found exactly once: %r" % old
    mutant_src = tmp_path / ("mutant_%s.c" % name)
    mutant_src.write_text(src.replace(old, new))
    lib = oracle.compile_oracle(str(mutant_src), str(tmp_path / ("mutant_%s.so" % name)))
    orc = oracle.Oracle(lib)
    caught = None
    for pin in ORDER:
        try:
            pins.ALL_PINS[pin](orc)
        except (AssertionError, RuntimeError) as e:   # RuntimeError: oracle self-check
            caught = pin
            break
    assert caught is not None, "planted mistake %s passed every pin" % name
