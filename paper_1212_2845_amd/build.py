"""Build the voxsim HIP library (libvoxsim.so) for gfx950, in-tree.

Every HIP source is compiled with hipcc for gfx950 only, with packed FP32
instructions disabled, and linked into one shared library that exports the
C ABI declared in include/voxsim.h.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libvoxsim.so")
SOURCES = ["vx_api.cpp", "vx_grad.cpp", "vx_batch.cpp", "vx_split.hip", "vx_fused.hip", "vx_collide.hip",
           "vx_adjoint.hip", "vx_adjoint_fused.hip", "vx_energy.hip", "vx_static.hip", "vx_statics.cpp"]
HEADERS = ["vx_types.hpp", "vx_device.hpp", "vx_launch.hpp", "vx_host.hpp", "vx_sim.hpp", "vx_adjoint.hpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-std=c++17", "-O3", "-fPIC", "--offload-arch=gfx950", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include")]


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    lang = ["-x", "hip"]
    cmd = [HIPCC] + COMMON + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def is_stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    srcs = [os.path.join(CSRC, f) for f in SOURCES + HEADERS] + [os.path.join(ROOT, "include", "voxsim.h")]
    return any(os.path.getmtime(p) > t for p in srcs)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
