"""Compile the CPU oracles into ``oracle/libfastref.so`` (detection) and
``oracle/liblkref.so`` (the Lucas-Kanade tracker): plain C, -O2, one thread."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def _compile(src_name: str, lib_name: str, verbose: bool) -> str:
    src = os.path.join(HERE, src_name)
    out = os.path.join(HERE, lib_name)
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(verbose: bool = False) -> str:
    _compile("lkref.c", "liblkref.so", verbose)
    return _compile("fastref.c", "libfastref.so", verbose)


if __name__ == "__main__":
    print(build(verbose=True))
