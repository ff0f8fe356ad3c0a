"""Build step for the CPU oracle (test infrastructure): one gcc call.

The flags keep the arithmetic plain: no fast-math, no FMA contraction, and
no -march=native, so a library built on one host also runs on another.
"""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


# Checks of the address and undefined-behaviour sanitizers, for the build the
# sanitizer test loads instead of the plain one (same arithmetic flags).
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
            "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, out: str | None = None, sanitize: bool = False) -> str:
    src = os.path.join(_HERE, "lddmm_oracle.c")
    out = out or os.path.join(_HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O1" if sanitize else "-O3", "-std=c11", "-Wall", "-Wextra",
           "-ffp-contract=off", "-fno-fast-math", *(SANITIZE if sanitize else []),
           "-fPIC", "-shared", "-o", tmp, src, "-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
