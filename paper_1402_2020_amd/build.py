"""Builds libbsm.so (the HIP library behind include/bsm.h) for gfx950.

Each source is compiled on its own (in parallel) with hipcc and the objects
are linked into a shared library next to this file.  Floating-point
contraction is off so that the host-side table and pattern arithmetic rounds
exactly as written; packed FP32 instructions are disabled for device code.
"""
import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbsm.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("BSM_OFFLOAD_ARCH", "gfx950")

SOURCES = ["bsm_host.cpp", "bsm_kernels.hip", "bsm_batch.cpp", "bsm_serve_core.cpp", "bsm_server.cpp",
           "bsm_noalloc.hip", "bsm_peaks.hip"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-result",
          "-I", os.path.join(HERE, "..", "include")]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src, verbose):
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    if src.endswith(".hip"):
        cmd = ["hipcc", "-x", "hip", *DEVICE, *COMMON, "-c", path, "-o", obj]
    else:
        cmd = ["hipcc", *COMMON, "-D__HIP_PLATFORM_AMD__", "-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    cmd = ["hipcc", *DEVICE, "-shared", "-fPIC", *objs, "-o", LIB + ".tmp", "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
