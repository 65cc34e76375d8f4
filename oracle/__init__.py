"""CPU oracle for the Wolff single-cluster update (Komura & Okabe, arXiv:1110.0899).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU product path
never imports it and shares no code with it.

The arithmetic lives in ``wolff_oracle.c`` (plain C, one core); this module
builds it with gcc and exposes it through ctypes with numpy arrays:

* ``philox(ctr, key)``          Philox4x32-10 (Salmon et al., SC'11)
* ``threshold(J, T)``           floor(p 2^32), p = 1 - exp(-2J/T)   (Section 2, step ii)
* ``seed_site(seed, t, N)``     step (i): the random site of update t
* ``init_spins(dim, L, seed)``  iid +-1 start
* ``observables(dim, L, S)``    (B, M) with E = -J B           (Section 5, "+ measurement")
* ``cluster(...)``              one cluster, steps (i)-(iv), membership mask
* ``run(...)``                  n updates, records (B, M, |C|) per update (steps (i)-(v))
* ``bond_draw(...)``            raw bond random number, for independent graph rebuilds
* ``potts_*``                   the q-state Potts extension (Section 6): threshold
                                1 - exp(-J/T), colours, new-colour draw, observables, run

``Oracle(path)`` wraps any build of the C file (the tests also build
deliberately broken copies to show that the pins catch them).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "wolff_oracle.c")
LIBRARY = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_default = None


def compile_oracle(src: str, out: str) -> str:
    """Compile one oracle source file with gcc into a shared library."""
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                           "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile oracle/wolff_oracle.c into oracle/liboracle.so (if stale)."""
    if force or not os.path.exists(LIBRARY) or os.path.getmtime(LIBRARY) < os.path.getmtime(SOURCE):
        compile_oracle(SOURCE, LIBRARY)
    return LIBRARY


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


class Oracle:
    """ctypes view of one compiled oracle library."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        u32, u64, i32, p = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
        lib.orc_philox4x32_10.argtypes = [p, p, p]
        lib.orc_philox4x32_10.restype = None
        lib.orc_threshold.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.orc_threshold.restype = u32
        lib.orc_seed_site.argtypes = [u64, u32, u64]
        lib.orc_seed_site.restype = u64
        lib.orc_init_spins.argtypes = [i32, i32, u64, p]
        lib.orc_init_spins.restype = None
        lib.orc_observables.argtypes = [i32, i32, p, p, p]
        lib.orc_observables.restype = None
        lib.orc_cluster.argtypes = [i32, i32, u32, u64, u32, p, p, p, p]
        lib.orc_cluster.restype = u64
        lib.orc_run.argtypes = [i32, i32, u32, u64, u32, u64, p, p]
        lib.orc_run.restype = i32
        lib.orc_bond_draw.argtypes = [u64, u32, u32, u32, i32]
        lib.orc_bond_draw.restype = u32
        self.has_potts = hasattr(lib, "orc_potts_run")
        if self.has_potts:
            lib.orc_potts_threshold.argtypes = [ctypes.c_double, ctypes.c_double]
            lib.orc_potts_threshold.restype = u32
            lib.orc_potts_init.argtypes = [i32, i32, i32, u64, p]
            lib.orc_potts_init.restype = None
            lib.orc_potts_new_colour.argtypes = [u64, u32, i32, i32]
            lib.orc_potts_new_colour.restype = i32
            lib.orc_potts_observables.argtypes = [i32, i32, i32, p, p, p]
            lib.orc_potts_observables.restype = None
            lib.orc_potts_run.argtypes = [i32, i32, i32, u32, u64, u32, u64, p, p]
            lib.orc_potts_run.restype = i32
        self.lib = lib
        self.path = path

    def philox(self, ctr, key) -> np.ndarray:
        c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(4))
        k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(2))
        out = np.zeros(4, dtype=np.uint32)
        self.lib.orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
        return out

    def threshold(self, J: float, T: float) -> int:
        return int(self.lib.orc_threshold(float(J), float(T)))

    def seed_site(self, seed: int, t: int, N: int) -> int:
        return int(self.lib.orc_seed_site(seed, t, N))

    def init_spins(self, dim: int, L: int, seed: int) -> np.ndarray:
        S = np.zeros(L ** dim, dtype=np.int8)
        self.lib.orc_init_spins(dim, L, seed, _ptr(S))
        return S

    def observables(self, dim: int, L: int, S: np.ndarray) -> tuple[int, int]:
        S = np.ascontiguousarray(S, dtype=np.int8)
        B = ctypes.c_int64()
        M = ctypes.c_int64()
        self.lib.orc_observables(dim, L, _ptr(S), ctypes.addressof(B), ctypes.addressof(M))
        return B.value, M.value

    def cluster(self, dim: int, L: int, thr: int, seed: int, t: int, S: np.ndarray):
        """Membership mask (uint8[N]), seed site s and its spin s0 for update t."""
        S = np.ascontiguousarray(S, dtype=np.int8)
        member = np.zeros(S.size, dtype=np.uint8)
        s = ctypes.c_uint64()
        s0 = ctypes.c_int()
        size = self.lib.orc_cluster(dim, L, thr, seed, t, _ptr(S), _ptr(member),
                                    ctypes.addressof(s), ctypes.addressof(s0))
        if size == 0:
            raise MemoryError("oracle cluster allocation failed")
        return member, int(s.value), int(s0.value)

    def run(self, dim: int, L: int, thr: int, seed: int, t0: int, n: int,
            S: np.ndarray) -> np.ndarray:
        """Run updates t0..t0+n-1 on S in place; returns int64[n, 3] = (B, M, |C|)."""
        assert S.dtype == np.int8 and S.flags["C_CONTIGUOUS"]
        rec = np.zeros((max(n, 0), 3), dtype=np.int64)
        if n == 0:
            return rec
        rc = self.lib.orc_run(dim, L, thr, seed, t0, n, _ptr(S), _ptr(rec))
        if rc == -1:
            raise MemoryError("oracle allocation failed")
        if rc != 0:
            raise RuntimeError("oracle consistency check failed (rc=%d)" % rc)
        return rec

    def bond_draw(self, seed: int, t: int, s: int, b: int, mu: int) -> int:
        return int(self.lib.orc_bond_draw(seed, t, s, b, mu))

    # ---- q-state Potts (Section 6's extension; readings in wolff_oracle.c)
    def potts_threshold(self, J: float, T: float) -> int:
        return int(self.lib.orc_potts_threshold(float(J), float(T)))

    def potts_init(self, dim: int, L: int, q: int, seed: int) -> np.ndarray:
        S = np.zeros(L ** dim, dtype=np.int8)
        self.lib.orc_potts_init(dim, L, q, seed, _ptr(S))
        return S

    def potts_new_colour(self, seed: int, t: int, q: int, s0: int) -> int:
        return int(self.lib.orc_potts_new_colour(seed, t, q, s0))

    def potts_observables(self, dim: int, L: int, q: int, S: np.ndarray) -> tuple[int, int]:
        S = np.ascontiguousarray(S, dtype=np.int8)
        B = ctypes.c_int64()
        M = ctypes.c_int64()
        self.lib.orc_potts_observables(dim, L, q, _ptr(S), ctypes.addressof(B), ctypes.addressof(M))
        return B.value, M.value

    def potts_run(self, dim: int, L: int, q: int, thr: int, seed: int, t0: int, n: int,
                  S: np.ndarray) -> np.ndarray:
        """Potts updates t0..t0+n-1 on the colours S in place; int64[n, 3] = (B, M, |C|)."""
        assert S.dtype == np.int8 and S.flags["C_CONTIGUOUS"]
        rec = np.zeros((max(n, 0), 3), dtype=np.int64)
        if n == 0:
            return rec
        rc = self.lib.orc_potts_run(dim, L, q, thr, seed, t0, n, _ptr(S), _ptr(rec))
        if rc == -1:
            raise MemoryError("oracle allocation failed")
        if rc != 0:
            raise RuntimeError("oracle consistency check failed (rc=%d)" % rc)
        return rec


def default() -> Oracle:
    global _default
    with _lock:
        if _default is None:
            _default = Oracle(build())
    return _default


def philox(ctr, key):
    return default().philox(ctr, key)


def threshold(J, T):
    return default().threshold(J, T)


def seed_site(seed, t, N):
    return default().seed_site(seed, t, N)


def init_spins(dim, L, seed):
    return default().init_spins(dim, L, seed)


def observables(dim, L, S):
    return default().observables(dim, L, S)


def cluster(dim, L, thr, seed, t, S):
    return default().cluster(dim, L, thr, seed, t, S)


def run(dim, L, thr, seed, t0, n, S):
    return default().run(dim, L, thr, seed, t0, n, S)


def bond_draw(seed, t, s, b, mu):
    return default().bond_draw(seed, t, s, b, mu)


def potts_threshold(J, T):
    return default().potts_threshold(J, T)


def potts_init(dim, L, q, seed):
    return default().potts_init(dim, L, q, seed)


def potts_new_colour(seed, t, q, s0):
    return default().potts_new_colour(seed, t, q, s0)


def potts_observables(dim, L, q, S):
    return default().potts_observables(dim, L, q, S)


def potts_run(dim, L, q, thr, seed, t0, n, S):
    return default().potts_run(dim, L, q, thr, seed, t0, n, S)
