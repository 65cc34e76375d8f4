"""ctypes binding of libwolff (include/wolff.h): argument marshalling only.

Every step of the Wolff update runs in the library's HIP kernels; this module
only converts Python values and numpy arrays to the C ABI.  torch is imported
first so that the library shares torch's HIP runtime in the process (and so
that torch streams can be handed to the library); it is used for nothing
else here.  If libwolff.so has not been built, loading fails loudly: there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

import torch  # noqa: F401  (one HIP runtime per process: torch's)

HERE = os.path.dirname(os.path.abspath(__file__))
# WOLFF_LIBRARY=stats loads the counting build (libwolff_stats.so), any other
# value is taken as a path; unset: libwolff.so
_CHOICE = os.environ.get("WOLFF_LIBRARY", "")
LIBRARY = (os.path.join(HERE, "libwolff_stats.so") if _CHOICE == "stats"
           else _CHOICE or os.path.join(HERE, "libwolff.so"))

OK, EINVAL, ENOMEM, EDEVICE, ERANGE, ESTATE, EABORTED = 0, -1, -2, -3, -4, -5, -6
NOT_MEASURED = -(2 ** 63)
PATH_AUTO, PATH_SINGLE, PATH_TEAM, PATH_LDS = 0, 1, 2, 3


class WolffError(RuntimeError):
    def __init__(self, code: int, where: str, message: str):
        super().__init__("%s failed (%d): %s" % (where, code, message))
        self.code = code


class Record(ctypes.Structure):
    _fields_ = [("bond_sum", ctypes.c_int64), ("mag", ctypes.c_int64), ("csize", ctypes.c_int64)]


class Info(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("L", ctypes.c_int32), ("n_sites", ctypes.c_uint64),
                ("J", ctypes.c_double), ("T", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("threshold", ctypes.c_uint32), ("path", ctypes.c_int32), ("t", ctypes.c_uint64),
                ("mag", ctypes.c_int64), ("bond_sum", ctypes.c_int64),
                ("records_pending", ctypes.c_uint64), ("q", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Buffers(ctypes.Structure):
    _fields_ = [("spins", ctypes.c_void_p), ("overflow", ctypes.c_void_p),
                ("records", ctypes.c_void_p), ("record_capacity", ctypes.c_uint64),
                ("team_queue", ctypes.c_void_p), ("t0", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


BUFFERS_KEEP_SPINS = 1


class JobDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("L", ctypes.c_int32), ("J", ctypes.c_double),
                ("T", ctypes.c_double), ("seed", ctypes.c_uint64), ("n_updates", ctypes.c_uint64),
                ("start", ctypes.c_int32), ("flags", ctypes.c_int32), ("q", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


JOB_UPDATE_ONLY = 1


class ServerStats(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_uint64), ("running", ctypes.c_uint64), ("done", ctypes.c_uint64),
                ("slots", ctypes.c_uint64), ("resident_bytes", ctypes.c_uint64),
                ("budget_bytes", ctypes.c_uint64), ("quanta", ctypes.c_uint64),
                ("updates", ctypes.c_uint64), ("added_spins", ctypes.c_uint64),
                ("gpu_ms", ctypes.c_double)]


JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED = 0, 1, 2, 3

# WOLFF_STAT_* counters of the counting build, in index order
STAT_NAMES = ["updates", "sites", "steps", "steps_narrow", "neighbour_reads", "philox", "claims",
              "read_bytes", "write_bytes", "atomic_bytes", "messages", "idle_polls", "cycles_grow",
              "cycles_idle", "cycles_expand", "cycles_publish", "steps_send", "cycles_send"]
STAT_COUNT = 18

RECORD_DTYPE = np.dtype([("bond_sum", np.int64), ("mag", np.int64), ("csize", np.int64)])

# name -> (restype, argtypes); every symbol declared in include/wolff.h
_P = ctypes.c_void_p
_U64 = ctypes.c_uint64
_I = ctypes.c_int
_D = ctypes.c_double
SIGNATURES = {
    "wolff_create": (_I, [_I, _I, _D, _D, _U64, ctypes.POINTER(_P)]),
    "wolff_create_potts": (_I, [_I, _I, _I, _D, _D, _U64, ctypes.POINTER(_P)]),
    "wolff_create_ex": (_I, [_I, _I, _D, _D, _U64, ctypes.POINTER(Buffers), ctypes.POINTER(_P)]),
    "wolff_run_noalloc": (_I, [_I, _I, _D, _D, _U64, _P, _U64, ctypes.c_uint32, _I, _U64, _P, _P]),
    "wolff_destroy": (_I, [_P]),
    "wolff_abort": (_I, [_P]),
    "wolff_run": (_I, [_P, _U64]),
    "wolff_observables": (_I, [_P, _P, _U64, ctypes.POINTER(_U64)]),
    "wolff_synchronize": (_I, [_P]),
    "wolff_get_info": (_I, [_P, ctypes.POINTER(Info)]),
    "wolff_get_spins": (_I, [_P, _P, _U64]),
    "wolff_set_spins": (_I, [_P, _P, _U64, _U64]),
    "wolff_set_measure": (_I, [_P, _I]),
    "wolff_set_stream": (_I, [_P, _P]),
    "wolff_set_path": (_I, [_P, _I, _I]),
    "wolff_set_graph": (_I, [_P, _I]),
    "wolff_set_lds_slab": (_I, [_P, ctypes.c_uint32]),
    "wolff_set_lds_tiles": (_I, [_P, _I]),
    "wolff_set_tiles": (_I, [_P, _I, _I]),
    "wolff_profile": (_I, [_P, _I]),
    "wolff_profile_read": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(_U64),
                                ctypes.POINTER(_D), ctypes.POINTER(_U64)]),
    "wolff_strerror": (ctypes.c_char_p, [_I]),
    "wolff_last_error": (ctypes.c_char_p, []),
    "wolff_batch_create": (_I, [ctypes.POINTER(JobDesc), _I, ctypes.POINTER(_P)]),
    "wolff_batch_destroy": (_I, [_P]),
    "wolff_batch_run": (_I, [_P, _U64]),
    "wolff_batch_records": (_I, [_P, _I, _P, _U64, ctypes.POINTER(_U64)]),
    "wolff_batch_progress": (_I, [_P, _I, ctypes.POINTER(_U64), ctypes.POINTER(_U64)]),
    "wolff_batch_get_spins": (_I, [_P, _I, _P, _U64]),
    "wolff_batch_set_measure": (_I, [_P, _I]),
    "wolff_batch_set_stream": (_I, [_P, _P]),
    "wolff_batch_set_graph": (_I, [_P, _I]),
    "wolff_batch_set_tiles": (_I, [_P, _I, _I]),
    "wolff_batch_set_lds": (_I, [_P, _I]),
    "wolff_batch_last_ms": (_I, [_P, ctypes.POINTER(_D)]),
    "wolff_batch_stats_read": (_I, [_P, _P, _I, _I]),
    "wolff_stats_read": (_I, [_P, _P, _I, _I]),
    "wolff_server_create": (_I, [_U64, _I, ctypes.POINTER(_P)]),
    "wolff_server_destroy": (_I, [_P]),
    "wolff_server_submit": (_I, [_P, ctypes.POINTER(JobDesc), ctypes.POINTER(_U64)]),
    "wolff_server_step": (_I, [_P, _D, ctypes.POINTER(_U64)]),
    "wolff_server_set_lds": (_I, [_P, _I]),
    "wolff_server_status": (_I, [_P, _U64, ctypes.POINTER(_I), ctypes.POINTER(_U64)]),
    "wolff_server_finished": (_I, [_P, _P, _U64, ctypes.POINTER(_U64)]),
    "wolff_server_take": (_I, [_P, _U64, _P, _U64, ctypes.POINTER(_U64)]),
    "wolff_server_get_stats": (_I, [_P, ctypes.POINTER(ServerStats)]),
}

_lib = None
_lock = threading.Lock()


def load(path: str = LIBRARY):
    """Load libwolff.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise FileNotFoundError(
                    "%s is missing: build it with `python -m paper_1110_0899_amd.build` "
                    "(there is no non-HIP fallback)" % path)
            lib = ctypes.CDLL(path)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def _check(rc: int, where: str):
    if rc != OK:
        msg = load().wolff_last_error().decode(errors="replace")
        raise WolffError(rc, where, msg)


def _stream_handle(stream) -> int | None:
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return int(stream.cuda_stream)
    return int(stream)


class Simulation:
    """One lattice: wolff_create / wolff_run / wolff_observables; with q >= 2
    the q-state Potts model (wolff_create_potts)."""

    def __init__(self, dim: int, L: int, J: float, T: float, seed: int, q: int = 0,
                 buffers: dict | None = None):
        """buffers: caller-owned device memory for wolff_create_ex, a dict
        with the raw device addresses "spins", "overflow", "records" (e.g.
        tensor.data_ptr()), "record_capacity", optional "team_queue", and
        optional "t0" (the spins buffer then already holds the state at
        update t0)."""
        lib = load()
        h = ctypes.c_void_p()
        if buffers is not None:
            keep = "t0" in buffers
            b = Buffers(int(buffers["spins"]), int(buffers["overflow"]), int(buffers["records"]),
                        int(buffers["record_capacity"]),
                        int(buffers["team_queue"]) if buffers.get("team_queue") else None,
                        int(buffers.get("t0", 0)), BUFFERS_KEEP_SPINS if keep else 0, 0)
            _check(lib.wolff_create_ex(dim, L, float(J), float(T), int(seed), ctypes.byref(b),
                                       ctypes.byref(h)), "wolff_create_ex")
        elif q:
            _check(lib.wolff_create_potts(dim, L, int(q), float(J), float(T), int(seed),
                                          ctypes.byref(h)), "wolff_create_potts")
        else:
            _check(lib.wolff_create(dim, L, float(J), float(T), int(seed), ctypes.byref(h)),
                   "wolff_create")
        self._h = h
        self.dim, self.L, self.J, self.T, self.seed, self.q = dim, L, J, T, seed, q
        self.n_sites = L ** dim

    def close(self):
        if getattr(self, "_h", None):
            load().wolff_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def run(self, n_updates: int):
        _check(load().wolff_run(self._h, int(n_updates)), "wolff_run")

    def observables(self, cap: int | None = None) -> np.ndarray:
        """Drain pending records: structured array (bond_sum, mag, csize)."""
        if cap is None:
            cap = self.info().records_pending
        out = np.zeros(int(cap), dtype=RECORD_DTYPE)
        n = _U64()
        _check(load().wolff_observables(self._h, out.ctypes.data if cap else None, int(cap),
                                        ctypes.byref(n)), "wolff_observables")
        return out[: n.value]

    def synchronize(self):
        _check(load().wolff_synchronize(self._h), "wolff_synchronize")

    def abort(self):
        """Stop the enqueued updates at the next update boundary (callable
        from another thread)."""
        _check(load().wolff_abort(self._h), "wolff_abort")

    def info(self) -> Info:
        inf = Info()
        _check(load().wolff_get_info(self._h, ctypes.byref(inf)), "wolff_get_info")
        return inf

    def spins(self) -> np.ndarray:
        S = np.zeros(self.n_sites, dtype=np.int8)
        _check(load().wolff_get_spins(self._h, S.ctypes.data, S.size), "wolff_get_spins")
        return S

    def set_spins(self, S: np.ndarray, t: int):
        S = np.ascontiguousarray(S, dtype=np.int8)
        _check(load().wolff_set_spins(self._h, S.ctypes.data, S.size, int(t)), "wolff_set_spins")

    def set_measure(self, on: bool):
        _check(load().wolff_set_measure(self._h, 1 if on else 0), "wolff_set_measure")

    def set_stream(self, stream=None):
        h = _stream_handle(stream)
        _check(load().wolff_set_stream(self._h, h), "wolff_set_stream")

    def set_path(self, path: int, workgroups: int = 0):
        _check(load().wolff_set_path(self._h, path, workgroups), "wolff_set_path")

    def set_lds_slab(self, slab_bits: int):
        _check(load().wolff_set_lds_slab(self._h, int(slab_bits)), "wolff_set_lds_slab")

    def set_lds_tiles(self, wg: int):
        _check(load().wolff_set_lds_tiles(self._h, int(wg)), "wolff_set_lds_tiles")

    def set_graph(self, chunk: int):
        _check(load().wolff_set_graph(self._h, int(chunk)), "wolff_set_graph")

    def set_tiles(self, wg: int, queue_entries: int):
        _check(load().wolff_set_tiles(self._h, int(wg), int(queue_entries)), "wolff_set_tiles")

    def stats(self, reset: bool = False) -> dict:
        """Counters of the counting build (libwolff_stats.so)."""
        out = (ctypes.c_uint64 * STAT_COUNT)()
        _check(load().wolff_stats_read(self._h, out, STAT_COUNT, 1 if reset else 0), "wolff_stats_read")
        return {k: int(out[i]) for i, k in enumerate(STAT_NAMES)}

    def profile(self, on: bool):
        _check(load().wolff_profile(self._h, 1 if on else 0), "wolff_profile")

    def profile_read(self) -> dict:
        g, gn, m, mn = _D(), _U64(), _D(), _U64()
        _check(load().wolff_profile_read(self._h, ctypes.byref(g), ctypes.byref(gn),
                                         ctypes.byref(m), ctypes.byref(mn)), "wolff_profile_read")
        return {"grow_ms": g.value, "grow_launches": gn.value,
                "measure_ms": m.value, "measure_launches": mn.value}


def run_noalloc(dim: int, L: int, J: float, T: float, seed: int, spins_ptr: int, n_updates: int,
                records_ptr: int, t0: int | None = None, measure: bool = True, stream=None):
    """wolff_run_noalloc on caller-owned device memory (raw addresses, e.g.
    tensor.data_ptr()); t0 given: the spins buffer holds the state at t0."""
    flags = BUFFERS_KEEP_SPINS if t0 is not None else 0
    _check(load().wolff_run_noalloc(dim, L, float(J), float(T), int(seed), int(spins_ptr),
                                    int(t0 or 0), flags, 1 if measure else 0, int(n_updates),
                                    int(records_ptr) if records_ptr else None,
                                    _stream_handle(stream)), "wolff_run_noalloc")


class Batch:
    """Many replicas advanced by one persistent launch per run()."""

    def __init__(self, jobs, start: int = 0, update_only: bool = False):
        """jobs: objects with dim, L, J, T, seed, n_updates (and q: 0 Ising,
        >= 2 Potts); start: 0 iid +-1 (colours) from each seed, +1 / -1
        ordered; update_only: no bond sum per update."""
        lib = load()
        arr = (JobDesc * len(jobs))()
        flags = JOB_UPDATE_ONLY if update_only else 0
        for i, j in enumerate(jobs):
            arr[i] = JobDesc(j.dim, j.L, float(j.J), float(j.T), int(j.seed), int(j.n_updates),
                             int(start), flags, int(getattr(j, "q", 0)), 0)
        h = ctypes.c_void_p()
        _check(lib.wolff_batch_create(arr, len(jobs), ctypes.byref(h)), "wolff_batch_create")
        self._h = h
        self.jobs = list(jobs)

    def close(self):
        if getattr(self, "_h", None):
            load().wolff_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def run(self, max_updates: int = 0):
        _check(load().wolff_batch_run(self._h, int(max_updates)), "wolff_batch_run")

    def records(self, job: int) -> np.ndarray:
        left, t = self.progress(job)
        cap = max(int(t), 1)
        out = np.zeros(cap, dtype=RECORD_DTYPE)
        n = _U64()
        _check(load().wolff_batch_records(self._h, job, out.ctypes.data, cap, ctypes.byref(n)),
               "wolff_batch_records")
        return out[: n.value]

    def progress(self, job: int):
        left, t = _U64(), _U64()
        _check(load().wolff_batch_progress(self._h, job, ctypes.byref(left), ctypes.byref(t)),
               "wolff_batch_progress")
        return left.value, t.value

    def spins(self, job: int) -> np.ndarray:
        j = self.jobs[job]
        S = np.zeros(j.L ** j.dim, dtype=np.int8)
        _check(load().wolff_batch_get_spins(self._h, job, S.ctypes.data, S.size),
               "wolff_batch_get_spins")
        return S

    def set_measure(self, on: bool):
        _check(load().wolff_batch_set_measure(self._h, 1 if on else 0), "wolff_batch_set_measure")

    def set_stream(self, stream=None):
        _check(load().wolff_batch_set_stream(self._h, _stream_handle(stream)),
               "wolff_batch_set_stream")

    def set_graph(self, on: bool):
        _check(load().wolff_batch_set_graph(self._h, 1 if on else 0), "wolff_batch_set_graph")

    def set_tiles(self, wg: int, queue_entries: int):
        _check(load().wolff_batch_set_tiles(self._h, wg, queue_entries), "wolff_batch_set_tiles")

    def set_lds(self, on: bool):
        _check(load().wolff_batch_set_lds(self._h, 1 if on else 0), "wolff_batch_set_lds")

    def stats(self, reset: bool = False) -> dict:
        """Counters of the counting build, summed over the replicas."""
        out = (ctypes.c_uint64 * STAT_COUNT)()
        _check(load().wolff_batch_stats_read(self._h, out, STAT_COUNT, 1 if reset else 0),
               "wolff_batch_stats_read")
        return {k: int(out[i]) for i, k in enumerate(STAT_NAMES)}

    def last_ms(self) -> float:
        ms = _D()
        _check(load().wolff_batch_last_ms(self._h, ctypes.byref(ms)), "wolff_batch_last_ms")
        return ms.value


class Server:
    """Continuous-batching request loop (wolff_server_*)."""

    def __init__(self, hbm_budget_bytes: int = 0, max_slots: int = 0):
        h = ctypes.c_void_p()
        _check(load().wolff_server_create(int(hbm_budget_bytes), int(max_slots), ctypes.byref(h)),
               "wolff_server_create")
        self._h = h
        self.n_updates = {}

    def close(self):
        if getattr(self, "_h", None):
            load().wolff_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, job, start: int = 0, update_only: bool = False) -> int:
        d = JobDesc(job.dim, job.L, float(job.J), float(job.T), int(job.seed), int(job.n_updates),
                    int(start), JOB_UPDATE_ONLY if update_only else 0, int(getattr(job, "q", 0)), 0)
        jid = _U64()
        _check(load().wolff_server_submit(self._h, ctypes.byref(d), ctypes.byref(jid)),
               "wolff_server_submit")
        self.n_updates[jid.value] = int(job.n_updates)
        return jid.value

    def set_lds(self, on: bool):
        _check(load().wolff_server_set_lds(self._h, 1 if on else 0), "wolff_server_set_lds")

    def step(self, quantum_ms: float) -> int:
        n = _U64()
        _check(load().wolff_server_step(self._h, float(quantum_ms), ctypes.byref(n)),
               "wolff_server_step")
        return n.value

    def status(self, job_id: int):
        st, done = ctypes.c_int(), _U64()
        _check(load().wolff_server_status(self._h, int(job_id), ctypes.byref(st), ctypes.byref(done)),
               "wolff_server_status")
        return st.value, done.value

    def finished(self, cap: int = 4096) -> list:
        ids = np.zeros(cap, dtype=np.uint64)
        n = _U64()
        _check(load().wolff_server_finished(self._h, ids.ctypes.data, cap, ctypes.byref(n)),
               "wolff_server_finished")
        return [int(v) for v in ids[: n.value]]

    def take(self, job_id: int) -> np.ndarray:
        cap = max(self.n_updates.get(job_id, 1), 1)
        out = np.zeros(cap, dtype=RECORD_DTYPE)
        n = _U64()
        _check(load().wolff_server_take(self._h, int(job_id), out.ctypes.data, cap, ctypes.byref(n)),
               "wolff_server_take")
        self.n_updates.pop(job_id, None)
        return out[: n.value]

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().wolff_server_get_stats(self._h, ctypes.byref(st)), "wolff_server_get_stats")
        return {name: getattr(st, name) for name, _ in ServerStats._fields_}
