"""The C ABI used from a plain C program (tests/c_abi/abi_check.c): no
Python, no torch; device memory from hipMalloc, a non-default stream.  The
program checks its results against direct DFT sums in double precision."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_2203_09384_amd")
ROCM = "/opt/rocm"


def build(out_dir):
    exe = os.path.join(out_dir, "abi_check")
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
           f"-I{ROCM}/include", f"-I{os.path.join(ROOT, 'include')}",
           os.path.join(HERE, "c_abi", "abi_check.c"), "-o", exe,
           f"-L{PKG}", "-lmifft", f"-L{ROCM}/lib", "-lamdhip64", "-lm",
           f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{ROCM}/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_c_program_builds_against_the_library(tmp_path):
    build(str(tmp_path))


@pytest.mark.gpu
def test_c_program_runs(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    exe = build(str(tmp_path))
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    assert "abi_check ok" in r.stdout
