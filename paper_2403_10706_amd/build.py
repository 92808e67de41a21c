"""Build librgp.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2403_10706_amd.build   (or call ``build()``)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "librgp.so")

SOURCES = ["api.cpp", "loss.hip", "pcg.hip", "ot.hip", "pyramid.hip", "lbfgs.hip", "lsq.hip",
           "admm.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # keep hipcc from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", CSRC,
]


# ROCTx (named host ranges for tracers), found at run time through the ROCm library directory
ROCM_LIB = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
LINK_LIBS = ["-L", ROCM_LIB, "-Wl,-rpath," + ROCM_LIB, "-lrocprofiler-sdk-roctx"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build librgp)")


def build(verbose: bool = False, jobs: int = 5, asan: bool = False) -> str:
    """Compile every source for gfx950 and link librgp.so next to this file.

    asan=True builds librgp_asan.so instead: the host code instrumented with AddressSanitizer
    (the device code is built as usual), for the host-side checks of the C ABI."""
    cc = hipcc()
    flags = list(HIPCC_FLAGS)
    lib = LIB
    if asan:
        flags += ["-O1", "-g", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address"]
        lib = os.path.join(HERE, "librgp_asan.so")
    with tempfile.TemporaryDirectory(prefix="rgp_build_") as tmp:
        objs = []
        procs = []
        for src in SOURCES:
            obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
            lang = ["-x", "hip"] if src.endswith(".cpp") else []
            cmd = [cc, *flags, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
            while len([p for _, p in procs if p.poll() is None]) >= jobs:
                procs[0][1].wait()
        for src, p in procs:
            out, _ = p.communicate()
            if p.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{out}")
            if verbose and out.strip():
                print(out)
        tmp_lib = lib + ".tmp"
        link_asan = ["-Xarch_host", "-fsanitize=address", "-shared-libasan"] if asan else []
        cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", *link_asan, *objs, *LINK_LIBS,
               "-o", tmp_lib]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
        os.replace(tmp_lib, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, asan="--asan" in sys.argv))
