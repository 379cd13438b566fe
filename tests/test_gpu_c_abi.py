"""The C ABI used from C: a program built against include/dirac.h and libdirac.so only (gcc,
the HIP runtime for device memory) applies the free-field operator to a point source and
compares every entry with the hopping term written out by hand; it also checks one refused
call (aliased output -> DIRAC_EINVAL with a message)."""
import os
import shutil
import subprocess

import pytest

from gpu_util import flush, need_gpu

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_2502_02490_amd")


def test_c_program_against_the_abi(tmp_path):
    need_gpu()
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "c_abi_check")
    cmd = ["gcc", "-std=c11", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
           os.path.join(HERE, "c_abi_check.c"), "-L" + PKG, "-ldirac", "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath," + PKG, "-Wl,-rpath,/opt/rocm/lib", "-lm", "-o", exe]
    subprocess.check_call(cmd)
    flush("[gpu] C ABI program")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    flush(out.stdout.strip())
    assert out.returncode == 0, out.stdout + out.stderr
    assert "C ABI OK" in out.stdout
