"""CPU sanitizer builds (no GPU): the FP64 oracle with address and
undefined-behaviour sanitizers (gcc), and libmpm's host-only logic (the
binomial schedule, error strings, the argument checks that return before any
HIP call) with the same sanitizers on the host side of a hipcc build.  Each
driver exits non-zero on a wrong result; a sanitizer report aborts it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (" ".join(cmd), r.stdout[-2000:], r.stderr[-4000:])
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "mpm_oracle.c"),
          os.path.join(HERE, "oracle_main.c"), "-lm", "-o", exe])
    r = _run([exe], env=ENV)
    assert "oracle sanitizer run: 0" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_library_host_logic_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "host_san")
    csrc = os.path.join(ROOT, "paper_1810_01054_amd", "csrc")
    _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include"),
          os.path.join(csrc, "mpm_kernels.hip"), os.path.join(csrc, "mpm_api.hip"),
          os.path.join(HERE, "host_main.cpp"), "-o", exe])
    r = _run([exe], env=ENV)
    assert "host sanitizer run: 0 problems" in r.stdout
