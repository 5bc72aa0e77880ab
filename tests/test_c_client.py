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


@pytest.mark.gpu
def test_c_client_on_the_gpu(tmp_path):
    """The whole path from C without PyTorch: workspace from hipMalloc, a HIP
    stream of the client's own, all 512 amplitudes of a 3x3 circuit in FP64
    and FP32 3M (normalisation and agreement checked by the client)."""
    import paper_1905_08394_amd as ps
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    lib_dir = os.path.dirname(ps.LIB_PATH)
    exe = tmp_path / "psim_gpu_client"
    cmd = ["gcc", "-std=c11", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"),
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c", "psim_gpu_client.c"), "-o", str(exe),
           "-L", lib_dir, "-lpsim", "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-lm",
           "-Wl,-rpath," + lib_dir, "-Wl,-rpath," + os.path.join(rocm, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout, flush=True)
    assert r.returncode == 0, r.stderr + r.stdout
    assert "c gpu client ok" in r.stdout
