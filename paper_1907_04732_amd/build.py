"""Build the HIP library liblbe.so for gfx950 (cross-compiles without a GPU).

Each source is compiled to an object of its own, in parallel, and the objects
are linked into liblbe.so.  The library carries the hash of the sources it
was built from (lbe_build_id); the Python binding refuses a library whose
hash differs from the sources beside it, so a stale build is never loaded.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
HEADER = os.path.join(ROOT, "include", "lbe.h")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblbe.so")
SOURCES = ["lbe_kernels.hip", "lbe_kernels_f32.hip", "lbe_mg.hip", "lbe_adjoint.hip",
           "lbe_noalloc.hip", "lbe_capi.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wall", "-Wno-unused-function",
]


def source_hash() -> str:
    """Hash of the library's sources: every file under csrc/ (names and
    contents, in name order) and the public header."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(f.encode())
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(fh.read())
    with open(HEADER, "rb") as fh:
        h.update(b"lbe.h")
        h.update(fh.read())
    return h.hexdigest()[:16]


def _compile(src: str, build_id: str, verbose: bool) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, f'-DLBE_BUILD_ID="{build_id}"', "-x", "hip", "-c",
           os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    build_id = source_hash()
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_id, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
