"""Builds libsfcdd.so (the C-ABI shared library) for gfx950 with hipcc.

Usage: python -m paper_2110_11211_amd.build_lib   (or call build()).
The library is written next to this file; it has no PyTorch dependency.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsfcdd.so")
SOURCES = ["setup.hip", "order.hip", "factor.hip", "trsv.hip", "apply.hip", "coarse_iter.hip", "sfcdd_api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    """Compiles every source and links the library; returns its path."""
    from concurrent.futures import ThreadPoolExecutor
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, "_build", src.replace(".hip", ".o"))
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        cmd = [HIPCC] + FLAGS[:-1] + ["-c", os.path.join(CSRC, src), "-o", obj]
        cmds.append([c for c in cmd if c != "-shared"])
        objs.append(obj)
    if verbose:
        for cmd in cmds:
            print(" ".join(cmd), flush=True)
    # the sources compile independently: one compiler process each
    with ThreadPoolExecutor(max_workers=min(len(cmds), 8)) as ex:
        for r in list(ex.map(lambda c: subprocess.run(c, check=False), cmds)):
            if r.returncode != 0:
                raise subprocess.CalledProcessError(r.returncode, r.args)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
