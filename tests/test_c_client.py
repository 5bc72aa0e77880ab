"""The C ABI from plain C: tests/c/psim_client.c compiled with gcc against
include/psim.h and linked to the built libpsim.so, run on the host (a
host-only plan; no device)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_c_client(tmp_path):
    import paper_1905_08394_amd as ps
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    lib_dir = os.path.dirname(ps.LIB_PATH)
    exe = tmp_path / "psim_client"
    cmd = ["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c", "psim_client.c"), "-o", str(exe), "-L", lib_dir, "-lpsim",
           "-Wl,-rpath," + lib_dir]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr + r.stdout
    assert "c client ok" in r.stdout
