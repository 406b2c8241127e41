"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
the CPU oracle (every public entry point, small models, overlaps 0-2) and the
decomposition planner and coefficient builder of the library (the host code
behind rbmc_plan_query and rbmc_model_create).  The drivers are in
tests/sanitize/; any sanitizer report (leaks included) fails the run.  GPU
code is not instrumented (the sanitizer flags are passed to the host
compilation only)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2309_05435_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out
    assert "runtime error" not in out and "AddressSanitizer" not in out, out
    assert "LeakSanitizer" not in out, out
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           "-ffp-contract=off", "-o", exe,
                           os.path.join(SAN, "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "rbmc_oracle.c"), "-lm"],
                          stderr=subprocess.DEVNULL)
    assert "oracle driver ok" in run(exe)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_planner_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "planner_san")
    subprocess.check_call([HIPCC, "-O1", "-g", "-std=c++17",
                           "-Xarch_host", "-fsanitize=address",
                           "-Xarch_host", "-fsanitize=undefined",
                           "-Xarch_host", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer",
                           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-o", exe,
                           os.path.join(SAN, "planner_driver.cpp"),
                           os.path.join(CSRC, "plan.cpp")], stderr=subprocess.DEVNULL)
    assert "planner driver ok" in run(exe)
