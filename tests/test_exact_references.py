"""The exact references that pin the oracle's 2D energy, pinned in turn.

The finite-torus partition function (Kaufman 1949, in the form of Ferdinand
& Fisher 1969) is checked against two constructions that share nothing with
it: the sum over all 2^16 states of the 4 x 4 torus, and the trace of the
L-th power of the row-to-row transfer matrix at L = 6, 8, 10.  Its derivative
<B> = d ln Z / dK (which the oracle's long L = 32 run is held to) is checked
against the enumerated Boltzmann average."""
import math

import numpy as np
import pytest

import exact_ising as ex
from paper_1110_0899_amd import workloads

K_VALUES = [0.25, 1.0 / workloads.TC_2D, 0.6]


def enumerated_lnZ(L, K):
    B, _ = ex.enumerate_states(2, L)
    shift = K * B.max()
    return float(shift + math.log(np.exp(K * B - shift).sum()))


@pytest.mark.parametrize("K", K_VALUES)
def test_kaufman_matches_enumeration_L4(K):
    exact = float(ex.kaufman_lnZ(4, K))
    assert abs(exact - enumerated_lnZ(4, K)) <= 1e-12 * abs(exact)


@pytest.mark.parametrize("L", [6, 8, 10])
@pytest.mark.parametrize("K", K_VALUES)
def test_kaufman_matches_transfer_matrix(L, K):
    exact = float(ex.kaufman_lnZ(L, K))
    assert abs(exact - ex.transfer_lnZ(L, K)) <= 1e-12 * abs(exact)


def test_transfer_matrix_matches_enumeration_L4():
    K = 1.0 / workloads.TC_2D
    assert abs(ex.transfer_lnZ(4, K) - enumerated_lnZ(4, K)) <= 1e-12 * enumerated_lnZ(4, K)


@pytest.mark.parametrize("K", K_VALUES)
def test_kaufman_mean_bond_sum_matches_enumeration(K):
    mom = ex.exact_moments(2, 4, K)
    assert abs(ex.kaufman_mean_B(4, K) - mom["B"]) <= 1e-10 * abs(mom["B"])
