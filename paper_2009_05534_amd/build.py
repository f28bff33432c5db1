"""Build the decoder library libldpc.so in-tree with hipcc for gfx950.

Each source compiles to its own object in parallel; the objects are then
linked into one shared library."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libldpc.so")
SOURCES = ["ldpc_api.hip", "decode_i8.hip", "decode_f16.hip", "nwms.hip", "batch.hip", "server.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off",
    # no packed fp32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _compile(src: str, obj: str, verbose: bool) -> None:
    cmd = [HIPCC, *FLAGS, "-c", "-o", obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def _stale(src: str, obj: str) -> bool:
    """An object is stale when it is missing or older than its source or
    any header of the source directory (or the public header)."""
    if not os.path.exists(obj):
        return True
    deps = [src, os.path.join(HERE, "..", "include", "ldpc.h")]
    deps += [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (or, with incremental=True, only those whose
    object in _build/ is stale) and link libldpc.so."""
    with tempfile.TemporaryDirectory(prefix="ldpc_build_") as tmpdir:
        objdir = tmpdir
        if incremental:
            objdir = os.path.join(HERE, "..", "_build")
            os.makedirs(objdir, exist_ok=True)
        objs = [os.path.join(objdir, s.replace(".hip", ".o")) for s in SOURCES]
        todo = [(s, o) for s, o in zip(SOURCES, objs)
                if not incremental or _stale(os.path.join(CSRC, s), o)]
        with cf.ThreadPoolExecutor(max_workers=max(1, len(todo))) as ex:
            futs = [ex.submit(_compile, os.path.join(CSRC, s), o, verbose) for s, o in todo]
            for f in futs:
                f.result()
        tmp = LIB + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, incremental="-i" in sys.argv)
    print(LIB)
