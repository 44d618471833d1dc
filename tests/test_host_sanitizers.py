"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the plan builder (compiled host-only with g++, driven by
tests/host/plan_driver.cpp) and the oracle (gcc, tests/host/orc_driver.c).
A sanitizer report fails the run (halt_on_error, non-zero exit)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
ENV.pop("LD_PRELOAD", None)
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-2000:], r.stderr[-4000:])
    return r


@pytest.mark.skipif(not os.path.exists("/opt/rocm/include/hip/hip_runtime.h"), reason="no HIP headers")
def test_plan_builder_sanitized(tmp_path):
    exe = tmp_path / "plan_driver"
    _run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
          "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2406_19920_amd", "csrc"),
          os.path.join(HOST, "plan_driver.cpp"),
          os.path.join(ROOT, "paper_2406_19920_amd", "csrc", "plan.cpp"), "-o", str(exe)])
    r = _run([str(exe)], env=ENV)
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert r.stdout.count("plan ") == 14


def test_oracle_sanitized(tmp_path):
    exe = tmp_path / "orc_driver"
    _run(["gcc", "-std=c99", *SAN, os.path.join(HOST, "orc_driver.c"),
          os.path.join(ROOT, "oracle", "orc.c"), "-o", str(exe), "-lm"])
    r = _run([str(exe)], env=ENV)
    assert "runtime error" not in r.stderr
    assert r.stdout.count("rel") == 48
