"""Exact references for the Ising model on small periodic lattices.

These are the independent pins for the oracle: they share no code with it and
use only textbook definitions.

* ``enumerate_states``   every configuration of a tiny lattice, with its bond
                         sum B = sum_i sum_mu S_i S_{i+e_mu} and M = sum_i S_i,
                         built from a numpy neighbour table (``np.roll``).
* ``exact_moments``      Boltzmann averages from the enumeration, weight
                         exp(K B), K = J/T (Hamiltonian of Section 2).
* ``kaufman_lnZ``        the exact partition function of the L x L torus
                         (Kaufman 1949, as written by Ferdinand & Fisher 1969).
* ``transfer_lnZ``       row-to-row transfer matrix on the L x L torus.
* ``kaufman_mean_B``     <B> = d lnZ / dK of the exact solution.
* ``active_bond_components``  connected components of the activated-bond
                         graph, by scipy's graph routine (no traversal code of
                         our own).
* ``block_mean_err``     mean and standard error from block averages.
"""
from __future__ import annotations

import math

import mpmath as mp
import numpy as np


def neighbour_tables(dim: int, L: int) -> list[np.ndarray]:
    """nb[mu][i] = index of i + e_mu (periodic); site index i = x + L*y (+ L^2 z)."""
    shape = (L,) * dim                     # C order: last axis is x (fastest)
    idx = np.arange(L ** dim).reshape(shape)
    tables = []
    for mu in range(dim):
        axis = dim - 1 - mu                # mu = 0 -> x -> last axis
        tables.append(np.roll(idx, -1, axis=axis).reshape(-1))
    return tables


def enumerate_states(dim: int, L: int) -> tuple[np.ndarray, np.ndarray]:
    """(B, M) for all 2^N states; state bit i set means S_i = -1."""
    N = L ** dim
    assert N <= 24
    states = np.arange(2 ** N, dtype=np.int64)
    spins = 1 - 2 * ((states[:, None] >> np.arange(N)[None, :]) & 1)
    M = spins.sum(axis=1)
    B = np.zeros(2 ** N, dtype=np.int64)
    for nb in neighbour_tables(dim, L):
        B += (spins * spins[:, nb]).sum(axis=1)
    return B, M


def bond_sum(dim: int, L: int, S: np.ndarray) -> int:
    S = S.astype(np.int64)
    return int(sum((S * S[nb]).sum() for nb in neighbour_tables(dim, L)))


def exact_moments(dim: int, L: int, K: float) -> dict:
    """Exact Boltzmann averages on the enumerated lattice at coupling K = J/T."""
    B, M = enumerate_states(dim, L)
    N = L ** dim
    w = np.exp(K * (B - B.max()).astype(np.float64))
    Z = w.sum()
    Mf = M.astype(np.float64)
    out = {
        "B": float((w * B).sum() / Z),
        "absM": float((w * np.abs(Mf)).sum() / Z),
        "M2": float((w * Mf ** 2).sum() / Z),
        "M4": float((w * Mf ** 4).sum() / Z),
        "N": N,
    }
    # joint distribution of (B, M)
    keys = B * (4 * N + 1) + (M + 2 * N)
    uniq, inv = np.unique(keys, return_inverse=True)
    prob = np.bincount(inv, weights=w) / Z
    out["dist_keys"] = uniq
    out["dist_prob"] = prob
    out["key_of"] = lambda b, m: b * (4 * N + 1) + (m + 2 * N)
    return out


def kaufman_lnZ(L: int, K, dps: int = 60):
    """ln Z of the L x L periodic square lattice, H = -J sum S_i S_j, K = J/T.

    Z = 1/2 (2 sinh 2K)^(L^2/2) (Z1 + Z2 + Z3 + Z4) with
    Z1 = prod_{r<L} 2 cosh(L g_{2r+1}/2),  Z2 = prod 2 sinh(L g_{2r+1}/2),
    Z3 = prod_{r<L} 2 cosh(L g_{2r}/2),    Z4 = prod 2 sinh(L g_{2r}/2),
    cosh g_l = cosh 2K coth 2K - cos(pi l / L) for l > 0 and
    g_0 = 2K + ln tanh K (signed).
    """
    with mp.workdps(max(dps, mp.mp.dps)):
        K = mp.mpf(K)
        c = mp.cosh(2 * K) * mp.coth(2 * K)

        def gamma(l):
            if l == 0:
                return 2 * K + mp.log(mp.tanh(K))
            return mp.acosh(c - mp.cos(mp.pi * l / L))

        Z1 = Z2 = Z3 = Z4 = mp.mpf(1)
        for r in range(L):
            go = gamma(2 * r + 1)
            ge = gamma(2 * r)
            Z1 *= 2 * mp.cosh(L * go / 2)
            Z2 *= 2 * mp.sinh(L * go / 2)
            Z3 *= 2 * mp.cosh(L * ge / 2)
            Z4 *= 2 * mp.sinh(L * ge / 2)
        return (mp.log(mp.mpf(1) / 2) + (mp.mpf(L * L) / 2) * mp.log(2 * mp.sinh(2 * K))
                + mp.log(Z1 + Z2 + Z3 + Z4))


def kaufman_mean_B(L: int, K, dps: int = 60) -> float:
    """<B> = d lnZ/dK on the L x L torus (so <E> = -J <B>)."""
    with mp.workdps(dps):
        return float(mp.diff(lambda k: kaufman_lnZ(L, k, dps), mp.mpf(K)))


def transfer_lnZ(L: int, K: float) -> float:
    """ln Z of the L x L torus from the row transfer matrix (L <= 10)."""
    rows = np.arange(2 ** L, dtype=np.int64)
    s = 1 - 2 * ((rows[:, None] >> np.arange(L)[None, :]) & 1)       # [2^L, L]
    intra = (s * np.roll(s, -1, axis=1)).sum(axis=1)                   # bonds within a row
    inter = s @ s.T                                                    # bonds between rows
    E = 0.5 * intra[:, None] + 0.5 * intra[None, :] + inter
    shift = K * E.max()
    T = np.exp(K * E - shift)
    ev = np.linalg.eigvalsh(T)
    # Z = Tr T^L = sum ev^L (T is symmetric)
    m = np.abs(ev).max()
    return float(L * (math.log(m) + shift) + math.log(np.sum((ev / m) ** L)))


def active_bond_components(dim: int, L: int, S: np.ndarray, active) -> np.ndarray:
    """Component labels of the graph whose edges are the bonds (b, mu) with
    active(b, mu) true and S_b == S_{b+e_mu}; computed by scipy."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    N = L ** dim
    rows, cols = [], []
    for mu, nb in enumerate(neighbour_tables(dim, L)):
        for b in range(N):
            k = int(nb[b])
            if S[b] == S[k] and active(b, mu):
                rows.append(b)
                cols.append(k)
    g = coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(N, N))
    _, labels = connected_components(g, directed=False)
    return labels


def block_mean_err(x: np.ndarray, nblocks: int = 40) -> tuple[float, float]:
    """Mean and standard error of a correlated series from block averages."""
    x = np.asarray(x, dtype=np.float64)
    n = (len(x) // nblocks) * nblocks
    blocks = x[:n].reshape(nblocks, -1).mean(axis=1)
    return float(x.mean()), float(blocks.std(ddof=1) / math.sqrt(nblocks))
