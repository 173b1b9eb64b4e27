"""The library's host code (level analysis, HEC and execution layouts,
factorizations, RAS layout) and the oracle's C code under AddressSanitizer
and UndefinedBehaviorSanitizer (tests/sanitize/host_checks.cpp).  Host only;
no GPU code is built with a sanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1606_00541_amd", "csrc")
FLAGS = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
INC = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="no host compiler")
def test_host_code_under_asan_and_ubsan(tmp_path):
    objs = []
    for src in (os.path.join(CSRC, "analysis.cpp"), os.path.join(CSRC, "factor.cpp"),
                os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp")):
        o = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run(["g++", "-std=c++17"] + FLAGS + INC + ["-c", src, "-o", o], check=True)
        objs.append(o)
    o = str(tmp_path / "orc.o")
    subprocess.run(["gcc", "-std=c99", "-ffp-contract=off"] + FLAGS +
                   ["-c", os.path.join(ROOT, "oracle", "orc.c"), "-o", o], check=True)
    objs.append(o)
    exe = str(tmp_path / "host_checks")
    subprocess.run(["g++", "-fsanitize=address,undefined", "-o", exe] + objs + ["-lm"], check=True)
    # verify_asan_link_order=0: the environment may preload other libraries
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "host checks passed" in r.stdout
