"""CPU tests of the serving layer: the C layouts of its structs, its
defaults, and the scheduler's arena and round planner (built with g++ from
the library's own header).  No device work."""

import ctypes
import subprocess

import pytest

from paper_1605_02164_amd import bfvec as B
from tests.helpers import ROOT

CSRC = f"{ROOT}/paper_1605_02164_amd/csrc"


def _layout(tmp_path, cname, ctype):
    fields = [n for n, _ in ctype._fields_]
    src = tmp_path / f"{cname}.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "bfvec.h"\n'
                   f"int main(void){{printf(\"%zu\", sizeof({cname}));" +
                   "".join(f'printf(" %zu", offsetof({cname}, {n}));' for n in fields) +
                   "return 0;}\n")
    exe = tmp_path / cname
    subprocess.run(["gcc", "-I", f"{ROOT}/include", str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    return got, [ctypes.sizeof(ctype)] + [getattr(ctype, n).offset for n in fields]


@pytest.mark.parametrize("cname", ["bf_server_config", "bf_request", "bf_request_status",
                                   "bf_server_stats"])
def test_server_struct_layouts(tmp_path, cname):
    got, want = _layout(tmp_path, cname, getattr(B, cname))
    assert got == want


def test_request_defaults():
    r = B.bf_request()
    B.lib().bf_request_init(ctypes.byref(r))
    assert (r.precision, r.center, r.N, r.pitch, r.arrival) == (B.BF_FP16, 1, 0, 0, 0.0)
    c = B.bf_server_config()
    B.lib().bf_server_config_init(ctypes.byref(c))
    assert (c.arena_bytes, c.max_active, c.streams, c.depth, c.quantum_us) == (0, 0, 0, 0, 0.0)


def test_null_arguments_rejected():
    L = B.lib()
    assert L.bf_server_create(None, None) == B.BF_EINVAL
    assert L.bf_server_submit(None, None, None) == B.BF_EINVAL
    assert L.bf_server_poll(None, 1, None) == B.BF_EINVAL
    assert L.bf_server_drain(None, 0.0) == B.BF_EINVAL
    assert L.bf_server_destroy(None) == B.BF_OK
    assert L.bf_server_clock(None) == 0.0


def test_scheduler_arena_and_planner(tmp_path):
    exe = tmp_path / "sched_check"
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-Werror", "-I", CSRC,
                    f"{ROOT}/tests/sched_check.cpp", "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    lines = out.stdout.split("\n")
    assert out.returncode == 0, out.stdout
    assert sum(l.startswith("PASS") for l in lines) == 5, out.stdout
