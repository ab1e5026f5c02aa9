"""Build librelax.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1405_0942_amd.build          # or: python paper_1405_0942_amd/build.py
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librelax.so")
SOURCES = ["stage.hip", "adjoint.hip", "control.hip", "stream.hip", "noalloc.hip", "relax.cpp"]
ARCH = os.environ.get("RELAX_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # no packed FP32 instructions in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{os.path.join(ROOT, 'include')}",
    f"-I{CSRC}",
]


def _compile(src: str, verbose: bool, tile_y: int) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(CSRC, f"{src}.ty{tile_y}.o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    # the 64 x 4 build's octilateral sweeps hold 94 KB of LDS, one 4-wave workgroup per CU, so
    # they cannot reach the two waves per SIMD their attribute asks for; the 64 x 8 build can
    quiet = ["-Wno-pass-failed"] if tile_y != 8 else []
    cmd = [HIPCC, *FLAGS, *quiet, f"-DRELAX_TILE_Y={tile_y}", *lang, "-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return obj


# The same library with 64 x 4 workgroup tiles instead of 64 x 8: built only so that a test
# can check that per-node results do not depend on the tile shape (an LDS race or a halo
# mistake would show there).
LIB_TY4 = os.path.join(HERE, "librelax_ty4.so")


def _build_one(path: str, tile_y: int, verbose: bool) -> str:
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, tile_y), SOURCES))
    tmp = path + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, path)
    for o in objs:
        os.remove(o)
    return path


def build(verbose: bool = False) -> str:
    _build_one(LIB_TY4, 4, verbose)
    return _build_one(LIB, 8, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
