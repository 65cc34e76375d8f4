"""Builds libwolff.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1110_0899_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBRARY = os.path.join(HERE, "libwolff.so")
# the counting build (-DWOLFF_STATS=1): the same kernels counting their work
# and the global-memory bytes they issue; for measurement, not for timing
STATS_LIBRARY = os.path.join(HERE, "libwolff_stats.so")
SOURCES = ["wolff_lib.hip"]
DEPENDS = ["wolff_lib.hip", "wolff_kernels.hip", "wolff_kernels.h", "wolff_device.h", "wolff_lds.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared", "-Wall",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # every global atomic here is issued by one lane (thread 0 or a wave's
    # leader, sums already taken with ballots); the compiler's wave-level
    # atomic combining would only add a scan and wait for the result at once
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
]


def _compile(out: str, extra: list, force: bool, verbose: bool) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    if not force and os.path.exists(out):
        newest = max(os.path.getmtime(os.path.join(CSRC, d)) for d in DEPENDS)
        newest = max(newest, os.path.getmtime(os.path.join(HERE, "..", "include", "wolff.h")))
        if os.path.getmtime(out) >= newest:
            return out
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + extra + ["-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise RuntimeError("hipcc failed building %s" % os.path.basename(out))
    os.replace(tmp, out)
    return out


def build(force: bool = True, verbose: bool = False, stats: bool = True) -> str:
    """Compile the library, and the counting build beside it (always when
    force is set, else when a source is newer)."""
    if stats:
        _compile(STATS_LIBRARY, ["-DWOLFF_STATS=1"], force, verbose)
    return _compile(LIBRARY, [], force, verbose)


if __name__ == "__main__":
    print(build(force=True, verbose=True))
