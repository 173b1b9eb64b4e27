"""Build the C part of the oracle (test infrastructure only).

The oracle is compiled with plain gcc at -O2 and -ffp-contract=off so that
no fused multiply-add changes its rounding; the CPU baseline of the benchmark
times a -O3 -march=native build of the same file made on the host it runs on
(build_native), whose results are identical.  The shared object lands next to
this file as ``liborc.so``.  The multithreaded level-scheduled CPU baseline
(``cpu_levels.c``, OpenMP) is built the same way into ``libcpulev.so``.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "orc.c")
LIB = os.path.join(HERE, "liborc.so")
SRC_OMP = os.path.join(HERE, "cpu_levels.c")
LIB_OMP = os.path.join(HERE, "libcpulev.so")


def _compile(src: str, lib: str, extra: list, force: bool) -> str:
    if (not force and os.path.exists(lib)
            and os.path.getmtime(lib) >= os.path.getmtime(src)):
        return lib
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-std=c99", "-Wall"] + extra + ["-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def build(force: bool = False) -> str:
    return _compile(SRC, LIB, [], force)


def build_native(dest_dir: str) -> str:
    """The same oracle compiled -O3 -march=native for the host it runs on
    (the CPU baseline's build), into dest_dir.  Contraction stays off and no
    reassociation is allowed, so its results equal the -O2 build's bit for
    bit."""
    os.makedirs(dest_dir, exist_ok=True)
    lib = os.path.join(dest_dir, "liborc_native.so")
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-march=native", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-std=c99", "-Wall", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def build_omp(force: bool = False) -> str:
    return _compile(SRC_OMP, LIB_OMP, ["-fopenmp"], force)


if __name__ == "__main__":
    print(build(force=True))
    print(build_omp(force=True))
