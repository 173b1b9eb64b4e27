"""Build libhec.so in-tree for gfx950.

Host-only translation units (analysis, factorization) are compiled with g++;
HIP translation units (kernels, C ABI, Krylov drivers) with hipcc for
--offload-arch=gfx950.  Packed FP32 instructions are disabled for all device
code.  Objects go to ``_build/``; the library lands next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhec.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

HOST_SRCS = ["analysis.cpp", "factor.cpp"]
HIP_SRCS = ["tri_kernels.hip", "krylov.hip", "refactor.hip", "capi.hip"]
HEADERS = ["hec_host.h", "hec_dev.h"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
HOST_FLAGS = COMMON + ["-ffp-contract=off", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include")]
HIP_FLAGS = COMMON + ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                      "-Wno-unused-command-line-argument"]


def _deps_mtime():
    paths = [os.path.join(CSRC, f) for f in HOST_SRCS + HIP_SRCS + HEADERS]
    paths.append(os.path.join(ROOT, "include", "hec.h"))
    return max(os.path.getmtime(p) for p in paths)


def up_to_date() -> bool:
    return os.path.exists(LIB) and os.path.getmtime(LIB) >= _deps_mtime()


def _stale(src: str, obj: str) -> bool:
    """An object older than its source or any header."""
    if not os.path.exists(obj):
        return True
    deps = [src] + [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(ROOT, "include", "hec.h")]
    return os.path.getmtime(obj) < max(os.path.getmtime(d) for d in deps)


def build(force: bool = True, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every translation unit and link libhec.so (always rebuilds
    when ``force``; with ``incremental`` only objects older than their
    sources or headers are recompiled)."""
    if not force and up_to_date():
        return LIB
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    objs = []
    for f in HOST_SRCS:
        o = os.path.join(BUILD, f + ".o")
        if not incremental or _stale(os.path.join(CSRC, f), o):
            jobs.append(["g++"] + HOST_FLAGS + ["-c", os.path.join(CSRC, f), "-o", o])
        objs.append(o)
    for f in HIP_SRCS:
        o = os.path.join(BUILD, f + ".o")
        if not incremental or _stale(os.path.join(CSRC, f), o):
            jobs.append([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, f), "-o", o])
        objs.append(o)
    procs = [(j, subprocess.Popen(j, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)) for j in jobs]
    failed = []
    for j, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append((j, text))
        elif verbose and text.strip():
            sys.stderr.write(text)
    if failed:
        msg = "\n\n".join(" ".join(j) + "\n" + t for j, t in failed)
        raise RuntimeError("libhec build failed:\n" + msg)
    tmp = LIB + ".tmp%d" % os.getpid()
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("libhec link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True, incremental="--incremental" in sys.argv))
