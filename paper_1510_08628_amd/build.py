"""Compile the gfx950 HIP library (libwarplda_hip.so) in-tree with hipcc.

Each source is compiled to an object of its own, in parallel, under
``_build/``; the objects are then linked into the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libwarplda_hip.so")
# (source, object name, extra flags): the per-M phase kernels are one source
# compiled once per M
SOURCES = [("wlda_kernels.hip", "wlda_kernels", [])] + \
    [("wlda_kernels_m.hip", f"wlda_kernels_m{m}", [f"-DWLDA_KM={m}"]) for m in (1, 2, 3, 4)] + \
    [(f, f.split(".")[0], []) for f in ("wlda_host.cpp", "wlda_foldin.hip", "wlda_encoder.hip",
                                        "wlda_server.cpp")]

# No FP contraction: the MH decisions are binary32 expressions that must round
# exactly as written.  Packed-FP32 instructions are disabled.
HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def sources():
    return [os.path.join(CSRC, s) for s in sorted({f for f, _, _ in SOURCES})]


def _compile(job, verbose: bool) -> str:
    src, name, extra = job
    obj = os.path.join(OBJ, name + ".o")
    cmd = ["hipcc", *HIPCC_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed on {src} ({name})")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(lambda j: _compile(j, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libwarplda_hip.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
