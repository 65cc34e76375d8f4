"""The C-ABI library builds, loads, exports every symbol include/wolff.h
declares, and rejects bad arguments before touching the GPU.  No compute
call is made here (this suite also runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1110_0899_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wolff.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wolff_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIBRARY):
        from paper_1110_0899_amd import build
        build.build(force=False)
    return binding.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("wolff_create", "wolff_run", "wolff_observables", "wolff_destroy"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    assert sorted(binding.SIGNATURES) == declared_functions()


def test_error_strings(lib):
    for code in (binding.OK, binding.EINVAL, binding.ENOMEM, binding.EDEVICE, binding.ERANGE,
                 binding.ESTATE, binding.EABORTED):
        assert lib.wolff_strerror(code)
    # every code has its own text
    texts = {lib.wolff_strerror(c) for c in range(-6, 1)}
    assert len(texts) == 7


@pytest.mark.parametrize("dim,L,J,T", [(1, 8, 1.0, 2.0), (4, 8, 1.0, 2.0), (2, 1, 1.0, 2.0),
                                       (2, 8, 0.0, 2.0), (2, 8, 1.0, 0.0), (2, 8, 1.0, float("nan")),
                                       (2, 8, float("inf"), 2.0), (2, 65536, 1.0, 2.0),
                                       (3, 1626, 1.0, 2.0)])
def test_create_rejects_bad_parameters(lib, dim, L, J, T):
    h = ctypes.c_void_p()
    rc = lib.wolff_create(dim, L, J, T, 1, ctypes.byref(h))
    assert rc == binding.EINVAL
    assert not h.value


def test_null_handles_are_rejected(lib):
    assert lib.wolff_run(None, 1) == binding.EINVAL
    assert lib.wolff_create(2, 8, 1.0, 2.0, 1, None) == binding.EINVAL
    assert lib.wolff_destroy(None) == binding.OK
    assert lib.wolff_batch_create(None, 0, None) == binding.EINVAL


@pytest.mark.parametrize("q", [0, 1, -3, 128, 1000])
def test_create_potts_rejects_bad_q(lib, q):
    # parameters are checked before any device call
    h = ctypes.c_void_p()
    assert lib.wolff_create_potts(2, 8, q, 1.0, 1.0, 1, ctypes.byref(h)) == binding.EINVAL
    assert not h.value


def test_noalloc_rejects_sizes_beyond_its_fixed_array(lib):
    # the size is checked before any device call
    for dim, L in ((2, 1025), (3, 102)):
        assert lib.wolff_run_noalloc(dim, L, 1.0, 2.0, 1, None, 0, 0, 1, 1, None, None) == binding.EINVAL
        assert b"scratch" in lib.wolff_last_error()


def job(**kw):
    j = binding.JobDesc(dim=2, L=16, J=1.0, T=2.269, seed=1, n_updates=10, start=0, flags=0, q=0)
    for k, v in kw.items():
        setattr(j, k, v)
    return j


@pytest.mark.parametrize("bad,code", [(dict(start=2), binding.EINVAL), (dict(start=-2), binding.EINVAL),
                                      (dict(flags=2), binding.EINVAL), (dict(q=1), binding.EINVAL),
                                      (dict(q=128), binding.EINVAL), (dict(dim=4), binding.EINVAL),
                                      (dict(L=1), binding.EINVAL), (dict(T=0.0), binding.EINVAL),
                                      (dict(n_updates=1 << 32), binding.ERANGE)])
def test_batch_create_rejects_bad_jobs(lib, bad, code):
    # every job is checked before any device call; the message names the job
    jobs = (binding.JobDesc * 2)(job(), job(**bad))
    h = ctypes.c_void_p()
    assert lib.wolff_batch_create(jobs, 2, ctypes.byref(h)) == code
    assert not h.value
    assert lib.wolff_last_error().startswith(b"job 1")


def test_batch_create_rejects_an_empty_list(lib):
    h = ctypes.c_void_p()
    jobs = (binding.JobDesc * 1)(job())
    assert lib.wolff_batch_create(jobs, 0, ctypes.byref(h)) == binding.EINVAL
    assert lib.wolff_batch_create(jobs, -1, ctypes.byref(h)) == binding.EINVAL
    assert lib.wolff_batch_create(jobs, 1, None) == binding.EINVAL


HANDLE_DESTROY = ("wolff_destroy", "wolff_batch_destroy", "wolff_server_destroy")


def null_args(argtypes):
    # a NULL handle first, then zeros and NULL pointers
    out = []
    for t in argtypes:
        if t in (ctypes.c_double,):
            out.append(0.0)
        elif t in (ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64):
            out.append(0)
        else:
            out.append(None)
    return out


def test_every_handle_call_rejects_a_null_handle(lib):
    # every entry point that takes a sim, batch or server handle checks it
    # first; destroying NULL is a no-op
    header = open(HEADER).read()
    takes_handle = set(re.findall(r"\b(wolff_\w+)\s*\(\s*(?:const\s+)?wolff_(?:sim|batch|server)\s*\*",
                                  re.sub(r"/\*.*?\*/", "", header, flags=re.S)))
    assert len(takes_handle) > 30
    for name in sorted(takes_handle):
        _, argtypes = binding.SIGNATURES[name]
        rc = getattr(lib, name)(*null_args(argtypes))
        assert rc == (binding.OK if name in HANDLE_DESTROY else binding.EINVAL), name


def test_server_rejects_bad_arguments_before_the_device(lib):
    assert lib.wolff_server_create(0, -1, ctypes.byref(ctypes.c_void_p())) == binding.EINVAL
    assert lib.wolff_server_create(0, 4, None) == binding.EINVAL
