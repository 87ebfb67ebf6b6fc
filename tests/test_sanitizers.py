"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the library's host-only C entry points (host.cpp: whitening, draws, order
rule, spatial taps, FP16 range rule) driven by tests/host_check.cpp, and the serving
scheduler's arena and round planner driven by tests/sched_check.cpp, both
built with g++ (no device code involved)."""

import shutil
import subprocess

import pytest

from tests.helpers import ROOT

CSRC = f"{ROOT}/paper_1605_02164_amd/csrc"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer", "-O1", "-g", "-std=c++17", "-Wall", "-Werror"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")


def _build_run(tmp_path, name, sources):
    exe = tmp_path / name
    subprocess.run(["g++", *SAN, "-I", f"{ROOT}/include", "-I", CSRC, *sources, "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True,
                         env={"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
                              "UBSAN_OPTIONS": "print_stacktrace=1"})
    return out


def test_host_entry_points_under_sanitizers(tmp_path):
    out = _build_run(tmp_path, "host_check",
                     [f"{ROOT}/tests/host_check.cpp", f"{CSRC}/host.cpp"])
    assert out.returncode == 0, out.stdout + out.stderr
    assert "runtime error" not in out.stderr and "ERROR: AddressSanitizer" not in out.stderr
    assert sum(l.startswith("PASS") for l in out.stdout.splitlines()) == 5, out.stdout


def test_scheduler_under_sanitizers(tmp_path):
    out = _build_run(tmp_path, "sched_check", [f"{ROOT}/tests/sched_check.cpp"])
    assert out.returncode == 0, out.stdout + out.stderr
    assert "runtime error" not in out.stderr and "ERROR: AddressSanitizer" not in out.stderr
    assert sum(l.startswith("PASS") for l in out.stdout.splitlines()) == 5, out.stdout
