"""Builds the HIP library libqilbm.so for gfx950 in-tree with hipcc.

Every call compiles from source (no up-to-date check). Sources: csrc/*.hip;
public header: include/qilbm.h at the repository root.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqilbm.so")
SOURCES = ["qilbm_kernels.hip", "qilbm_capi.hip", "qilbm_adjoint.hip", "qilbm3d.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions (v_pk_*_f32) anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("command failed: " + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    return res


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        for res in ex.map(_run, cmds):
            if verbose and (res.stdout or res.stderr):
                print(res.stdout + res.stderr, file=sys.stderr)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    build_c_example(objdir)
    return LIB


C_EXAMPLE_SRC = os.path.join(os.path.dirname(HERE), "tests", "c", "abi_example.c")
C_EXAMPLE = os.path.join(HERE, "_build", "abi_example")


def build_c_example(objdir: str) -> str:
    """A plain C11 program that uses the library through include/qilbm.h
    only (host compiler, HIP runtime API for device memory)."""
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    _run(["gcc", "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__",
          f"-I{rocm}/include", f"-I{os.path.join(os.path.dirname(HERE), 'include')}",
          C_EXAMPLE_SRC, "-o", C_EXAMPLE, f"-L{HERE}", "-lqilbm", f"-L{rocm}/lib",
          "-lamdhip64", "-lm", f"-Wl,-rpath,{rocm}/lib", "-Wl,-rpath,$ORIGIN/.."])
    return C_EXAMPLE


if __name__ == "__main__":
    print(build(verbose=True))
