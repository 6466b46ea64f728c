"""Build the HIP library libmeg.so, the native driver meg_bench and the
counter-calibration copy meg_copy, in-tree for gfx950.

    python -m paper_2012_10469_amd.build

The library is a plain shared object with the C ABI of include/meg.h; the
Python binding loads it with ctypes.  meg_bench links it (rpath $ORIGIN) and
runs the benchmark workload without Python, for profilers.  Packed-FP32
instruction forms are disabled for every HIP translation unit.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmeg.so")
DRIVER = os.path.join(HERE, "meg_bench")
COPY = os.path.join(HERE, "meg_copy")
ARCH = os.environ.get("MEG_OFFLOAD_ARCH", "gfx950")

SOURCES = ["meg_api.hip", "meg_serve.hip", "meg_exact.hip"]
HEADERS = ["meg_device.hpp", "meg_small.hpp", "meg_kernels.hpp", "meg_host.hpp"]

HIP_FLAGS = [
    "-O3",
    "-std=c++17",
    f"--offload-arch={ARCH}",
    "-fPIC",
    "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile libmeg.so (always recompiles) and return its path."""
    cmd = [hipcc(), *HIP_FLAGS, "-I", os.path.join(ROOT, "include")]
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    # rocBLAS for the plain GEMMs of the exact-MEG baseline's matrix exponential
    cmd += ["-o", tmp, "-L", "/opt/rocm/lib", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with exit code {res.returncode}")
    os.replace(tmp, LIB)
    # host-only driver: no device code of its own
    dcmd = [hipcc(), "-O2", "-std=c++17", "-Wno-unused-result", "-I", os.path.join(ROOT, "include"),
            os.path.join(CSRC, "meg_bench.cpp"), "-L", HERE, "-lmeg", "-Wl,-rpath,$ORIGIN", "-o", DRIVER + ".tmp"]
    if verbose:
        print(" ".join(dcmd), flush=True)
    res = subprocess.run(dcmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc (meg_bench) failed with exit code {res.returncode}")
    os.replace(DRIVER + ".tmp", DRIVER)
    # calibration copy for the traffic counters (own device code, no library)
    ccmd = [hipcc(), "-O2", "-std=c++17", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
            "-packed-fp32-ops", "-Wno-unused-result", os.path.join(CSRC, "meg_copy.cpp"), "-o", COPY + ".tmp"]
    if verbose:
        print(" ".join(ccmd), flush=True)
    res = subprocess.run(ccmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc (meg_copy) failed with exit code {res.returncode}")
    os.replace(COPY + ".tmp", COPY)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
