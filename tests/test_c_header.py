"""include/lbm.h as a C99 caller sees it: a C program that includes the
header with warnings as errors, links liblbm.so and calls it.  Without a GPU
only the host-side calls run (lbm_create then reports LBM_ENODEV); the GPU
variant of the test steps a small box."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2002_02503_amd")


def _build(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("needs gcc")
    if not os.path.exists(os.path.join(PKG, "liblbm.so")):
        pytest.fail("liblbm.so is not built (run __graft_entry__.build())")
    exe = str(tmp_path / "c_abi_example")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", f"-I{os.path.join(ROOT, 'include')}",
           os.path.join(ROOT, "tests", "c_abi_example.c"), f"-L{PKG}", "-llbm", f"-Wl,-rpath,{PKG}",
           "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return exe


def test_header_compiles_as_c99_and_host_calls_work(tmp_path):
    exe = _build(tmp_path)
    env = dict(os.environ, HIP_VISIBLE_DEVICES="")  # host-side calls only
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert "c abi example" in r.stdout


@pytest.mark.gpu
def test_c_caller_steps_a_box(tmp_path):
    exe = _build(tmp_path)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert "after 10 steps" in r.stdout
