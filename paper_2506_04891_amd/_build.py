"""Builds libtqsim.so in-tree for gfx950 (hipcc for the kernels and ABI, g++ for
the host planner)."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libtqsim.so")

HIP_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        lines = [ln for ln in r.stdout.splitlines() if "packed-fp32-ops" not in ln]
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + "\n".join(lines[-80:]))


def _stale(obj, sources):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(src) > t for src in sources)


def build(verbose=False, if_changed=False):
    """Compile the planner and the HIP translation unit, link libtqsim.so.
    if_changed: skip the HIP compile when its object is newer than every file
    it includes (for quick rebuilds after host-only changes)."""
    os.makedirs(BUILD, exist_ok=True)
    planner_o = os.path.join(BUILD, "planner.o")
    tqsim_o = os.path.join(BUILD, "tqsim.o")
    inc = ["-I", CSRC, "-I", INCLUDE]
    _run(["g++", "-O2", "-fPIC", "-std=c++17", "-Wall", *inc, "-c",
          os.path.join(CSRC, "planner.cpp"), "-o", planner_o])
    hip_srcs = [os.path.join(CSRC, f) for f in ("tqsim.hip", "kernels.hip", "plan.h", "planner.h")]
    hip_srcs.append(os.path.join(INCLUDE, "tqsim.h"))
    if not if_changed or _stale(tqsim_o, hip_srcs):
        _run(["hipcc", *HIP_FLAGS, *inc, "-c", os.path.join(CSRC, "tqsim.hip"), "-o", tqsim_o])
    tmp = LIB + ".tmp"
    _run(["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", tqsim_o, planner_o, "-o", tmp])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    import sys
    build(verbose=True, if_changed="--if-changed" in sys.argv)
