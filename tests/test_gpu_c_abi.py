"""The C ABI from a plain C program (tests/c/abi_example.c, built by the
package build next to the library): no Python or PyTorch in the process
that drives the GPU. It runs a 64x64 droplet in FP64 and FP32 and a 32^3
droplet through the three-dimensional header (FP64 periodic, FP32 with
walls and gravity) and checks the phi total (FP64 to 1e-12, FP32 exactly)."""
import os
import subprocess

import pytest

from paper_1507_03521_amd import build

pytestmark = pytest.mark.gpu


def test_c_program_drives_the_library():
    exe = build.C_EXAMPLE
    assert os.path.exists(exe), "run the package build first (it compiles the C example)"
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(res.stdout, res.stderr, flush=True)
    assert res.returncode == 0
    assert "abi example ok" in res.stdout
