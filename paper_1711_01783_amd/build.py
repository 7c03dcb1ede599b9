"""Builds the decoder library ``libmetbp.so`` in-tree for gfx950.

    python paper_1711_01783_amd/build.py

(Run as a file, not as ``-m``: importing the package loads the library, which
may be missing or stale before the build.)

hipcc cross-compiles for gfx950 without a GPU.  Packed FP32 instructions are
disabled for all device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmetbp.so")
SOURCES = ["met_code.cpp", "met_decode.hip", "met_wbp.hip", "met_batched.hip", "met_mdr.hip"]
ARCH = os.environ.get("MET_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)
    if verbose and err.strip():
        print(err, file=sys.stderr)


def build(verbose: bool = False) -> str:
    """Compiles every source to an object in parallel, then links the library
    (written to a temporary name and moved into place)."""
    from concurrent.futures import ThreadPoolExecutor

    tag = "%d" % os.getpid()
    objs = [os.path.join(CSRC, s + ".%s.o" % tag) for s in SOURCES]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    tmp = LIB + ".tmp" + tag
    try:
        with ThreadPoolExecutor(max_workers=len(SOURCES)) as pool:
            jobs = [pool.submit(_run, [hipcc(), *FLAGS, *inc, "-c", os.path.join(CSRC, s), "-o", o], verbose)
                    for s, o in zip(SOURCES, objs)]
            for j in jobs:
                j.result()
        _run([hipcc(), *FLAGS, "-shared", *objs, "-o", tmp], verbose)
        os.replace(tmp, LIB)
    finally:
        for f in objs + [tmp]:
            if os.path.exists(f):
                os.remove(f)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
