"""Build the CPU oracle library liboracle.so with gcc (C99 + OpenMP, no FMA contraction).

The oracle is test infrastructure: this script only builds the checker.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-Wall",
          "-Wno-unused-function", "-Wno-unused-macros"]


def build(verbose: bool = False, sanitize: bool = False, out: str | None = None) -> str:
    extra = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"] \
        if sanitize else []
    objs = []
    for tag, defs in (("r", []), ("z", ["-DORACLE_COMPLEX"])):
        obj = os.path.join(os.path.dirname(out) if out else HERE, f"oracle_{tag}{'_asan' if sanitize else ''}.o")
        cmd = ["gcc", *CFLAGS, *extra, *defs, "-c", SRC, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        objs.append(obj)
    if out is None:
        out = LIB if not sanitize else os.path.join(HERE, "liboracle_asan.so")
    cmd = ["gcc", "-shared", "-fopenmp", *extra, *objs, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    for o in objs:
        os.remove(o)
    return out


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--asan" in sys.argv))
