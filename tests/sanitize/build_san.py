"""Sanitizer builds for the CPU test suite.

* The oracle (plain C) with a driver program, by gcc with AddressSanitizer
  and UndefinedBehaviorSanitizer.
* The voxsim library with its host code instrumented the same way (the
  device code is built as usual for gfx950) and linked with a driver
  program that calls the C ABI without a GPU.

The two programs share no code.  Each build is skipped when the executable
is newer than every source it is made from.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "_build")
sys.path.insert(0, ROOT)

from paper_1212_2845_amd import build as vxbuild  # noqa: E402

HOST_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
              "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all"]


def _fresh(exe, sources):
    return os.path.exists(exe) and all(os.path.getmtime(exe) >= os.path.getmtime(s) for s in sources)


def build_oracle_program():
    exe = os.path.join(OUT, "oracle_drive")
    srcs = [os.path.join(HERE, "oracle_drive.c"), os.path.join(ROOT, "oracle", "vx_oracle.c"),
            os.path.join(ROOT, "oracle", "vx_oracle.h")]
    if _fresh(exe, srcs):
        return exe
    os.makedirs(OUT, exist_ok=True)
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-Wall", "-Wextra",
           "-I" + os.path.join(ROOT, "oracle"), srcs[0], srcs[1], "-lm", "-o", exe]
    subprocess.check_call(cmd)
    return exe


def _compile(src, out_dir):
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = [vxbuild.HIPCC] + vxbuild.COMMON + HOST_FLAGS + ["-x", "hip", "-c", os.path.join(vxbuild.CSRC, src),
                                                            "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    return obj


def build_host_program():
    exe = os.path.join(OUT, "host_drive")
    driver = os.path.join(HERE, "host_drive.cpp")
    srcs = ([os.path.join(vxbuild.CSRC, f) for f in vxbuild.SOURCES + vxbuild.HEADERS] +
            [os.path.join(ROOT, "include", "voxsim.h"), driver])
    if _fresh(exe, srcs):
        return exe
    objdir = os.path.join(OUT, "host")
    os.makedirs(objdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(vxbuild.SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, objdir), vxbuild.SOURCES))
    drv = os.path.join(objdir, "host_drive.o")
    subprocess.check_call([vxbuild.HIPCC, "-std=c++17", "-I" + os.path.join(ROOT, "include")] + HOST_FLAGS +
                          ["-c", driver, "-o", drv])
    subprocess.check_call([vxbuild.HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
                           "-Xarch_host", "-fsanitize=undefined", "-o", exe] + objs + [drv])
    return exe


if __name__ == "__main__":
    print(build_oracle_program())
    print(build_host_program())
