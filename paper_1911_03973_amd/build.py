"""Build libfem.so (HIP for gfx950) in-tree with hipcc.

Every HIP source is compiled for gfx950 only, with packed-FP32 instructions
disabled, into paper_1911_03973_amd/_lib/libfem.so.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libfem.so")
OBJ_DIR = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["plan.cpp", "plan_check.cpp", "local.hip", "apply.hip", "pcg.hip", "batch.hip", "api.hip", "batch_api.hip", "unet.hip",
           "fcg.hip", "iterate.hip", "mg.hip"]

COMMON = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    "-I" + CSRC,
    "-I" + os.path.join(ROOT, "include"),
]
HIP_FLAGS = [
    "--offload-arch=" + ARCH,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast",
]


# Sources of the solver's element pass: a profile of that pass is current only
# while these files are unchanged.
ELEMENT_PASS_SOURCES = ("plan.h", "plan.cpp", "common.h", "chunk.h", "kernels.h", "solver.h", "pcg.hip")


def sources_hash(names=ELEMENT_PASS_SOURCES) -> str:
    """Short SHA-256 over the named csrc files (name and content, in the given order)."""
    import hashlib

    h = hashlib.sha256()
    for n in names:
        h.update(n.encode())
        with open(os.path.join(CSRC, n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _compile(src: str, verbose: bool) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    obj = os.path.join(OBJ_DIR, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [HIPCC, "-x", "hip", *COMMON, *HIP_FLAGS, "-c", path, "-o", obj]
    else:
        cmd = [HIPCC, *COMMON, "-x", "c++", "-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source and link libfem.so; returns its path."""
    os.makedirs(OUT_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


# Host-only sources of the planner: plain C++, also built on their own with the
# address and undefined-behaviour sanitizers (g++, no HIP).
HOST_SOURCES = ("plan.cpp", "plan_check.cpp")
SANITIZED_LIB = os.path.join(OBJ_DIR, "libplan_san.so")


def build_host_sanitized(verbose: bool = False) -> str:
    """The host planner (fem_plan_check_host, fem_plan_check_host_p2) with
    -fsanitize=address,undefined, for the sanitizer tests; returns its path."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    tmp = SANITIZED_LIB + ".tmp"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-shared", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-I" + CSRC,
           "-I" + os.path.join(ROOT, "include"), *[os.path.join(CSRC, f) for f in HOST_SOURCES], "-o", tmp,
           "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, SANITIZED_LIB)
    return SANITIZED_LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
