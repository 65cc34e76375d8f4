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
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.wolff_strerror(code)


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
