"""AddressSanitizer and UndefinedBehaviorSanitizer runs on the CPU.

The oracle runs every entry point over small lattices (setters, channels,
contact with and without candidate overflow, instability, degenerate
inputs); the library's host side runs creation, validation, the per-bond
constants, timestep and surface list, state marshalling and every setter
without a GPU.  Any out-of-bounds access, leak or undefined behaviour
aborts the program with a report.
"""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "sanitize"))

import build_san  # noqa: E402

ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "Sanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers():
    assert "all scenarios passed" in _run(build_san.build_oracle_program())


@pytest.mark.skipif(not os.path.exists(build_san.vxbuild.HIPCC), reason="hipcc not found")
def test_host_side_under_sanitizers():
    assert "all scenarios passed" in _run(build_san.build_host_program())
