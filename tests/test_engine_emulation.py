"""Host logic of the fused pass engine, checked on the CPU.

tests/engine_emu/emu.cpp is compiled against the library's own host-side
source (the pass scheduler and the register-layout planner) and replays the
planned passes with a CPU model of the kernels' data movement, comparing
states, expectation values and gradients with an op-by-op reference.  It
needs hipcc (host compilation only) and the built library; no GPU.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_2508_13615_amd")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def emu_binary(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    lib = os.path.join(PKG, "libsv.so")
    if not os.path.exists(lib):
        pytest.skip("libsv.so not built")
    out = str(tmp_path_factory.mktemp("emu") / "emu")
    cmd = [HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
           os.path.join(HERE, "engine_emu", "emu.cpp"), "-o", out, "-L", PKG, "-lsv", f"-Wl,-rpath,{PKG}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return out


def test_planner_and_data_movement_match_reference(emu_binary):
    r = subprocess.run([emu_binary, "quick"], capture_output=True, text=True, timeout=600)
    print(r.stdout[-4000:])
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-2000:]
    assert "all ok (0 errors)" in r.stdout
