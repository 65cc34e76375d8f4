"""Binder-ratio estimator (CPU) and the batched Binder scan against exact
enumeration on tiny lattices (GPU)."""
import math

import numpy as np
import pytest

from paper_1110_0899_amd import studies


def test_binder_ratio_limits():
    # ordered: |M| fixed -> U = 2/3; Gaussian M -> U -> 0
    assert studies.binder_ratio(np.array([5, -5, 5, 5, -5])) == pytest.approx(2.0 / 3.0)
    rng = np.random.default_rng(1)
    g = rng.normal(size=400_000)
    assert abs(studies.binder_ratio(g)) < 0.01
    # two-point distribution {0, a} with equal weight: <M^2> = a^2/2, <M^4> = a^4/2 -> U = 1/3
    assert studies.binder_ratio(np.array([0.0, 3.0] * 10)) == pytest.approx(1.0 / 3.0)


def test_binder_error_scales_like_one_over_sqrt_n():
    rng = np.random.default_rng(2)
    e1 = studies.binder_error(rng.normal(size=20_000))
    e2 = studies.binder_error(rng.normal(size=320_000))
    assert 2.5 < e1 / e2 < 6.5        # sqrt(16) = 4


def test_crossing_interpolation():
    rows = [{"L": 8, "T": 1.0, "U": 0.60}, {"L": 8, "T": 2.0, "U": 0.40},
            {"L": 16, "T": 1.0, "U": 0.64}, {"L": 16, "T": 2.0, "U": 0.30}]
    # d(T) = U8 - U16: -0.04 at 1, +0.10 at 2 -> zero at 1 + 0.04/0.14
    assert studies.crossing(rows, 8, 16) == pytest.approx(1.0 + 0.04 / 0.14)
    assert studies.crossing(rows[:1] + rows[2:3], 8, 16) is None


@pytest.mark.gpu
@pytest.mark.parametrize("dim,L,temps", [(2, 4, (1.8, 2.269185314213022, 3.0)), (3, 2, (3.0, 4.5, 6.0))])
def test_batched_binder_matches_enumeration(dim, L, temps):
    import exact_ising
    from paper_1110_0899_amd import binding
    binding.load()
    print("case binder dim=%d L=%d" % (dim, L), flush=True)
    rows = studies.binder_scan(dim, [L], list(temps), discard=500, measure=60_000)
    for r in rows:
        ex = exact_ising.exact_moments(dim, L, 1.0 / r["T"])
        U = 1.0 - ex["M4"] / (3.0 * ex["M2"] ** 2)
        assert abs(r["U"] - U) < 5.0 * r["U_err"] + 1e-3, (r, U)
        assert r["bond_per_site"] == pytest.approx(ex["B"] / ex["N"], abs=0.05)
