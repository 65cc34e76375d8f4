"""MI355X (gfx950) Wolff single-cluster Monte Carlo for the 2D square and 3D
simple-cubic Ising model (Komura & Okabe, arXiv:1110.0899).

The compute path is libwolff.so (HIP kernels behind the C ABI in
include/wolff.h); ``binding`` is its ctypes wrapper, ``workloads`` holds the
seeded synthetic inputs.  Importing the package loads nothing; the library is
loaded on first use of ``Simulation`` or ``Batch``.
"""
import importlib

__all__ = ["Simulation", "Batch", "WolffError"]


def __getattr__(name):
    if name in __all__:
        return getattr(importlib.import_module(__name__ + ".binding"), name)
    raise AttributeError(name)
