"""Build libsubcull.so for gfx950 with hipcc (no torch extension machinery).

    python -m paper_2305_08343_amd.build             # libsubcull.so
    python -m paper_2305_08343_amd.build --sanitize  # libsubcull_san.so: host code under
                                                     # AddressSanitizer + UBSan (device code as usual)

The sanitized library is for CPU-side checks of the host code (argument
checks, the BVH builder, the 4-wide collapse, the codebook): load it with
SUBCULL_LIB pointing at it and the clang ASan runtime preloaded.

Flags that matter for reproducibility: -ffp-contract=off (no fused
multiply-add, so every float32 product rounds before it is added),
correctly rounded float32 division, denormals kept, and packed-fp32
instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsubcull.so")
SOURCES = ["api.cpp", "bvh.cpp", "codebook.cpp", "codebook.hip", "kernels_build.hip", "kernels_trace.hip",
           "kernels_trace_checked.hip", "placement.hip", "raysort.hip", "bvh4.cpp", "noalloc.hip"]
ARCH = os.environ.get("SUBCULL_ARCH", "gfx950")

COMMON = [
    "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
    "-ffp-contract=off", "-fno-fast-math",
]
DEVICE = [
    f"--offload-arch={ARCH}", "-fno-gpu-flush-denormals-to-zero",
    "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; ROCm is required to build libsubcull")
    return exe


# host-side sanitizers only: each -fsanitize= applies to the host compilation (-Xarch_host)
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]
SAN_DIR = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(HERE, "libsubcull_san.so")


def _compile(src: str, sanitize: bool = False) -> str:
    obj = os.path.join(SAN_DIR if sanitize else OUT_DIR, os.path.basename(src) + ".o")
    cmd = [hipcc()] + COMMON + (SANITIZE if sanitize else [])
    if src.endswith(".hip"):
        cmd += DEVICE + ["-x", "hip"]
    cmd += ["-I", os.path.join(HERE, "..", "include"), "-c", os.path.join(SRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


PROBE_SRC = os.path.join(HERE, "probes", "valu_rate.hip")
PROBE_BIN = os.path.join(HERE, "probes", "valu_rate")


def build_probe(verbose: bool = False) -> str:
    """The vector-ALU issue-rate probe (a stand-alone program, not part of the library)."""
    cmd = [hipcc()] + COMMON + DEVICE + ["-o", PROBE_BIN, PROBE_SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if verbose:
        print("built", PROBE_BIN)
    return PROBE_BIN


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out_dir, lib = (SAN_DIR, SAN_LIB) if sanitize else (OUT_DIR, LIB)
    os.makedirs(out_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, sanitize), SOURCES))
    tmp = lib + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if sanitize:
        cmd += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
    if "--sanitize" not in sys.argv[1:]:
        build_probe(verbose=True)
    sys.exit(0)
