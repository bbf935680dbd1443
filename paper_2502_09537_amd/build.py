"""Build libkgs.so in-tree: HIP kernels for gfx950 with hipcc, the host side
with the host C++ compiler, linked by hipcc.

    python -m paper_2502_09537_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libkgs.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall",
    # every fused multiply-add is written out: all kernels round identically
    "-ffp-contract=off",
    # keep packed fp32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]
HOST_FLAGS = [
    "-O2", "-fPIC", "-std=c++17", "-Wall", "-pthread", "-D__HIP_PLATFORM_AMD__",
    "-I", os.path.join(ROCM, "include"), "-I", INCLUDE, "-I", CSRC,
]


def sources():
    hip = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    cpp = sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp"))
    return hip, cpp


def build(verbose: bool = False) -> str:
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    cxx = shutil.which("g++") or "c++"
    os.makedirs(BUILD_DIR, exist_ok=True)
    hip, cpp = sources()
    jobs = []
    objs = []
    for f in hip:
        obj = os.path.join(BUILD_DIR, f + ".o")
        objs.append(obj)
        jobs.append([hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, f), "-o", obj])
    for f in cpp:
        obj = os.path.join(BUILD_DIR, f + ".o")
        objs.append(obj)
        jobs.append([cxx, *HOST_FLAGS, "-c", os.path.join(CSRC, f), "-o", obj])
    procs = [(cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
             for cmd in jobs]
    failed = []
    for cmd, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # the host pass of hipcc does not know the packed-fp32 feature; harmless
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l]
        if p.returncode != 0:
            failed.append((cmd, "\n".join(lines)))
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        msg = "\n\n".join(" ".join(c) + "\n" + t for c, t in failed)
        raise RuntimeError("libkgs build failed:\n" + msg)
    tmp = LIB + ".tmp"
    link = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
            "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lrocprofiler-sdk-roctx", "-pthread",
            "-Wl,--no-undefined"]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("libkgs link failed:\n" + " ".join(link) + "\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
