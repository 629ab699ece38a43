"""Build the fd3d HIP library (gfx950) in-tree: paper_2112_15071_amd/libfd3d.so.

Each translation unit of csrc/ is compiled on its own (in parallel), then linked."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
SOURCES = ["runtime.hip", "forward.hip", "gradient.hip", "batch.hip", "born.hip"]
LIB = os.path.join(PKG, "libfd3d.so")
OBJ = os.path.join(PKG, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # no packed FP32 instructions in any kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-add fusion decided per source expression, never across statements, so
    # that the same expression rounds the same way in every kernel variant
    "-ffp-contract=on",
    "-Wall",
    "-Wno-unused-function",
]


def _run(cmd, verbose, what):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for " + what)


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every HIP source of the library and link it (always recompiles)."""
    os.makedirs(OBJ, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmds.append(([HIPCC, *FLAGS, *inc, "-c", "-o", obj, os.path.join(CSRC, src)], src))
    workers = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        for f in [ex.submit(_run, cmd, verbose, what) for cmd, what in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose, "the link")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
