"""Build the CPU oracle shared libraries (plain C, gcc).  Test infrastructure.

libckks_oracle.so      the checker: one thread (the OpenMP pragmas are ignored)
libckks_oracle_omp.so  the same source built with -fopenmp, for timing the
                       oracle on all host cores (limb loops in parallel)
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ckks_oracle.c")
LIB = os.path.join(HERE, "libckks_oracle.so")
LIB_OMP = os.path.join(HERE, "libckks_oracle_omp.so")
FLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra"]


def _build_one(out: str, extra: list, verbose: bool) -> str:
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", *FLAGS, *extra, SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    _build_one(LIB, ["-Wno-unknown-pragmas"], verbose)
    _build_one(LIB_OMP, ["-fopenmp"], verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
