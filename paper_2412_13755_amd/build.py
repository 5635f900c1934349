"""Builds libtpcreco.so in place with hipcc for gfx950 only.

    python -m paper_2412_13755_amd.build

Each source compiles to an object with its own flags (the neighbour search
needs -ffp-contract=off so that no multiply-add is fused), then the objects
link into one shared library next to this file.  Packed-FP32 instruction
selection is disabled for all device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtpcreco.so")

SOURCES = {
    "tpc_api.hip": [],
    "tpc_neighbours.hip": ["-ffp-contract=off"],
    "tpc_ca_seed.hip": [],
    "tpc_fit.hip": [],
    "tpc_adjoint.hip": [],
    "tpc_persistent.hip": [],
    "tpc_follow.hip": [],
    "tpc_rans.hip": [],
    "tpc_ctf.hip": [],
    "tpc_fit_ms.hip": [],
    "tpc_merge.hip": [],
    "tpc_refit.hip": [],
    "tpc_nb_skip.hip": ["-ffp-contract=off"],
}

COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Wall",
          "-fno-gpu-flush-denormals-to-zero",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(HERE, "..", "include")]


# TPC_SANITIZE=1 builds libtpcreco_san.so instead: the host code (argument
# checks, workspace carving, launch setup) instrumented with clang's
# AddressSanitizer and UndefinedBehaviorSanitizer; device code is built as
# usual.  Load it with clang's ASan runtime preloaded.
SANITIZE = os.environ.get("TPC_SANITIZE", "") == "1"
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
if SANITIZE:
    BUILD = os.path.join(HERE, "_build_san")
    LIB = os.path.join(HERE, "libtpcreco_san.so")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str, extra) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [hipcc(), *COMMON, *extra, *(SAN_HOST if SANITIZE else []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on %s" % src)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda kv: _compile(*kv), SOURCES.items()))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", *(SAN_HOST if SANITIZE else []), *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
