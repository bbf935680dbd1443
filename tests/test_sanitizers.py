"""CPU-only AddressSanitizer + UndefinedBehaviorSanitizer runs: the C oracle
(tests/sanitize/oracle_driver.c) and the host side of libkgs's C ABI
(tests/sanitize/abi_driver.cpp against the library's host sources, linked
with the HIP objects of the last build).  Every call the ABI driver makes is
refused or answered before the library touches a device."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")

pytestmark = pytest.mark.slow


def _run(exe, tmp_path):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=ENV, cwd=tmp_path)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-3000:] + r.stderr[-3000:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    cmd = ["gcc", *SAN, "-std=c11", "-ffp-contract=off", "-fopenmp", "-o", exe,
           os.path.join(ROOT, "oracle", "kgs_oracle.c"),
           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=600)
    _run(exe, tmp_path)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_abi_host_side_under_asan_and_ubsan(tmp_path):
    from paper_2502_09537_amd import build

    hip, cpp = build.sources()
    objs = [os.path.join(build.BUILD_DIR, f + ".o") for f in hip]
    if not all(os.path.exists(o) for o in objs):
        build.build()
    rocm = build.ROCM
    exe = str(tmp_path / "abi_san")
    cmd = ["g++", *SAN, "-std=c++17", "-pthread", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(rocm, "include"), "-I", build.INCLUDE, "-I", build.CSRC,
           "-o", exe, os.path.join(ROOT, "tests", "sanitize", "abi_driver.cpp"),
           *[os.path.join(build.CSRC, f) for f in cpp], *objs,
           "-L", os.path.join(rocm, "lib"), "-Wl,-rpath," + os.path.join(rocm, "lib"),
           "-lamdhip64", "-lrocprofiler-sdk-roctx"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-3000:]
    _run(exe, tmp_path)
