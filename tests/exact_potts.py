"""Exact references for the q-state Potts model on tiny periodic lattices,
from the textbook definition H = -J sum_<ij> delta(s_i, s_j): every colouring
is enumerated (numpy, base-q digits), with the record observables
B = sum_i sum_mu (q delta(s_i, s_{i+e_mu}) - 1) and M = sum_i (q delta(s_i, 0) - 1)."""
from __future__ import annotations

import numpy as np

from exact_ising import neighbour_tables


def enumerate_states(dim: int, L: int, q: int):
    """(B, M) of all q^N colourings; colouring c has digit i = colour of site i."""
    N = L ** dim
    codes = np.arange(q ** N, dtype=np.int64)
    cols = np.empty((q ** N, N), dtype=np.int8)
    for i in range(N):
        cols[:, i] = (codes // q ** i) % q
    B = np.zeros(q ** N, dtype=np.int64)
    for nb in neighbour_tables(dim, L):
        B += np.where(cols == cols[:, nb], q - 1, -1).sum(axis=1)
    M = np.where(cols == 0, q - 1, -1).sum(axis=1).astype(np.int64)
    return B, M


def exact_moments(dim: int, L: int, q: int, K: float) -> dict:
    """Boltzmann averages at K = J/T; the weight of a colouring is
    exp(K * number of satisfied bonds) = exp(K (B + d N) / q)."""
    B, M = enumerate_states(dim, L, q)
    N = L ** dim
    e = K * (B + dim * N) / q
    w = np.exp(e - e.max())
    Z = w.sum()
    Mf = M.astype(np.float64)
    return {"B": float((w * B).sum() / Z), "M2": float((w * Mf ** 2).sum() / Z),
            "M4": float((w * Mf ** 4).sum() / Z), "N": N}
