"""Seeded synthetic workloads shared by the GPU path's tests, the benchmark and
the oracle-side checks.

Holds no part of the method's arithmetic: only the lattice sizes,
temperatures, seeds and update counts of each workload, and the generators of
the multi-replica and job-stream lists (numpy PCG64, fixed seeds).

The lattices and temperatures follow the paper's experiments: the square
lattice at T_c/J = 2/ln(1+sqrt 2) = 2.269... and the simple-cubic lattice at
T_c/J ~ 4.51 (Section 5), periodic boundaries (Section 2), and the paper's
sizes L = 512..4096 (2D) and 64..256 (3D) (Tables 1 and 2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict

import numpy as np

TC_2D = 2.0 / math.log(1.0 + math.sqrt(2.0))     # 2.269185314213022
T_3D = 4.511528                                   # simple-cubic critical temperature used here
J = 1.0


@dataclass(frozen=True)
class Job:
    dim: int
    L: int
    T: float
    seed: int
    n_updates: int
    J: float = J
    arrival_s: float = 0.0
    q: int = 0                  # 0: Ising; q >= 2: q-state Potts

    @property
    def n_sites(self) -> int:
        return self.L ** self.dim

    def as_dict(self) -> dict:
        return asdict(self)


# Single-lattice workloads: (name, dim, L, T, seed, thermalisation, measured updates)
C1 = dict(name="2d_L32_Tc", dim=2, L=32, T=TC_2D, seed=1, n_therm=0, n_meas=10_000)
C2 = dict(name="2d_L4096_Tc", dim=2, L=4096, T=TC_2D, seed=2, n_therm=1_000, n_meas=10_000)
C3 = dict(name="3d_L256_Tc", dim=3, L=256, T=T_3D, seed=3, n_therm=1_000, n_meas=10_000)


def c4_jobs(n_updates: int = 10_000) -> list[Job]:
    """Mixed replica set: 256 square-lattice replicas with L in {64..1024} and
    T ~ U[2.0, 2.6], plus 64 simple-cubic replicas with L in {32, 64, 128} and
    T ~ U[4.3, 4.7]; replica r has seed 0x40000000 + r."""
    rng = np.random.Generator(np.random.PCG64(4))
    jobs = []
    L2 = rng.choice([64, 128, 256, 512, 1024], size=256)
    T2 = rng.uniform(2.0, 2.6, size=256)
    L3 = rng.choice([32, 64, 128], size=64)
    T3 = rng.uniform(4.3, 4.7, size=64)
    r = 0
    for L, T in zip(L2, T2):
        jobs.append(Job(2, int(L), float(T), 0x40000000 + r, n_updates))
        r += 1
    for L, T in zip(L3, T3):
        jobs.append(Job(3, int(L), float(T), 0x40000000 + r, n_updates))
        r += 1
    return jobs


def potts_tc_2d(q: int) -> float:
    """Critical temperature of the square-lattice q-state Potts model (J = 1):
    T_c = 1 / ln(1 + sqrt q) (self-duality)."""
    return 1.0 / math.log(1.0 + math.sqrt(q))


def same_shape_jobs(dim: int, L: int, n_replicas: int, n_updates: int, q: int = 0,
                    T: float | None = None) -> list[Job]:
    """n_replicas copies of one lattice (at its critical temperature unless
    T is given) with per-replica seeds 0x48000000 + r; q >= 2: Potts."""
    if T is None:
        T = (potts_tc_2d(q) if q else TC_2D) if dim == 2 else T_3D
    return [Job(dim, L, T, 0x48000000 + r, n_updates, q=q) for r in range(n_replicas)]


def c5_stream(n_jobs: int = 2000, rate_per_s: float = 100.0, seed: int = 5) -> list[Job]:
    """Poisson job stream: half square-lattice jobs with L log-uniform in
    [64, 4096], half simple-cubic with L log-uniform in [32, 256];
    T = T_c (1 + U[-0.02, 0.02]); update counts log-uniform in [1e2, 1e4];
    exponential inter-arrival times at the given rate; job j has seed
    0x50000000 + j."""
    rng = np.random.Generator(np.random.PCG64(seed))
    jobs = []
    t = 0.0
    for j in range(n_jobs):
        t += float(rng.exponential(1.0 / rate_per_s))
        dim = 2 if rng.random() < 0.5 else 3
        if dim == 2:
            L = int(round(math.exp(rng.uniform(math.log(64), math.log(4096)))))
            T = TC_2D * (1.0 + rng.uniform(-0.02, 0.02))
        else:
            L = int(round(math.exp(rng.uniform(math.log(32), math.log(256)))))
            T = T_3D * (1.0 + rng.uniform(-0.02, 0.02))
        n = int(round(math.exp(rng.uniform(math.log(1e2), math.log(1e4)))))
        jobs.append(Job(dim, L, float(T), 0x50000000 + j, n, arrival_s=t))
    return jobs
