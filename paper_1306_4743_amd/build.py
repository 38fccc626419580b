"""Builds libeik.so (the HIP solver behind include/eik.h) in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libeik.so")
# The same solver with every write-back of a visit through an atomic minimum (a race check:
# its results must equal libeik.so's).
MINSTORE_LIB = os.path.join(HERE, "libeik_minstore.so")
SOURCES = ["eik_api.hip", "eik_kernels.hip"]
PROBE_LIB = os.path.join(HERE, "libeik_probe.so")
PROBE_SOURCES = ["eik_probe.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off: plain float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    f"-I{os.path.join(ROOT, 'include')}",
]


def _compile(out: str, sources, verbose: bool, extra=()) -> str:
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, *extra, "-o", tmp, *[os.path.join(CSRC, s) for s in sources]]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    """Compile the solver into paper_1306_4743_amd/libeik.so, its min-store debug build into
    libeik_minstore.so and the bandwidth probes into libeik_probe.so (always recompiles, the two
    solver builds in parallel); returns the solver library's path."""
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(3) as ex:
        jobs = [ex.submit(_compile, PROBE_LIB, PROBE_SOURCES, verbose),
                ex.submit(_compile, MINSTORE_LIB, SOURCES, verbose, ("-DEIK_DEBUG_MIN_STORES",)),
                ex.submit(_compile, LIB, SOURCES, verbose)]
        for j in jobs:
            j.result()
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
