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


PASS_UNITS = ("pass_f32_fwd", "pass_f32_bwd", "pass_f64_fwd", "pass_f64_bwd")


def build(verbose=False, if_changed=False):
    """Compile the planner and the HIP translation units (the host API and one
    unit per element type and direction of the tile-pass kernels, in
    parallel), link libtqsim.so.
    if_changed: skip a HIP compile whose object is newer than every file it
    includes (for quick rebuilds after host-only changes)."""
    os.makedirs(BUILD, exist_ok=True)
    planner_o = os.path.join(BUILD, "planner.o")
    inc = ["-I", CSRC, "-I", INCLUDE]
    # files each unit includes: the pass units see the kernels and the plan
    # layout only; the host API unit also the planner and the public header
    pass_deps = [os.path.join(CSRC, f) for f in ("kernels.hip", "plan.h", "pass_launch.h", "pass_tu.inc")]
    host_deps = pass_deps + [os.path.join(CSRC, "planner.h"), os.path.join(INCLUDE, "tqsim.h")]
    units = ["tqsim", *PASS_UNITS]
    procs, objs = [], []
    for u in units:
        src = os.path.join(CSRC, u + ".hip")
        obj = os.path.join(BUILD, u + ".o")
        objs.append(obj)
        deps = host_deps if u == "tqsim" else pass_deps
        if if_changed and not _stale(obj, [src, *deps]):
            continue
        cmd = ["hipcc", *HIP_FLAGS, *inc, "-c", src, "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    _run(["g++", "-O2", "-fPIC", "-std=c++17", "-Wall", *inc, "-c",
          os.path.join(CSRC, "planner.cpp"), "-o", planner_o])
    for cmd, pr in procs:
        out, _ = pr.communicate()
        if pr.returncode != 0:
            lines = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln]
            raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + "\n".join(lines[-80:]))
    tmp = LIB + ".tmp"
    _run(["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", *objs, planner_o, "-o", tmp])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    import sys
    build(verbose=True, if_changed="--if-changed" in sys.argv)
