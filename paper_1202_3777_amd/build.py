"""Build the in-tree HIP library ``libjt.so`` for gfx950.

Host C++ (planner, C ABI) is compiled with g++ against the HIP runtime
headers; the kernels are compiled with hipcc for gfx950 only.  Packed FP32
instructions are disabled in the device code generation.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libjt.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
ARCH = "gfx950"

HOST_SRCS = ["jt_plan.cpp", "jt_api.cpp"]
DEVICE_SRCS = ["jt_kernels.hip", "jt_paper.hip", "jt_bn.hip", "jt_scratch.hip"]
DEVICE_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    subprocess.check_call(cmd)


def sources():
    return [os.path.join(CSRC, s) for s in HOST_SRCS + DEVICE_SRCS] + [
        os.path.join(CSRC, "jt_internal.h"), os.path.join(CSRC, "jt_plan.h"), os.path.join(CSRC, "jt_api_internal.h"),
        os.path.join(ROOT, "include", "jt.h")]


def build(verbose: bool = False, defines=(), out: str = LIB, build_dir: str = BUILD) -> str:
    """Compile and link the library; ``defines`` are extra -D flags for both
    compilers (tuning constants), ``out`` the library path."""
    os.makedirs(build_dir, exist_ok=True)
    dfl = [f"-D{d}" for d in defines]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    for s in HOST_SRCS:
        o = os.path.join(build_dir, s.replace(".cpp", ".o"))
        _run(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__",
              "-I", os.path.join(ROCM, "include")] + dfl + inc + ["-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in DEVICE_SRCS:
        o = os.path.join(build_dir, s.replace(".hip", ".o"))
        _run([HIPCC] + DEVICE_FLAGS + dfl + inc + ["-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    tmp = out + ".tmp"
    # librocprofiler-sdk-roctx: the host-side trace ranges around propagations and sweeps
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs +
         ["-L", os.path.join(ROCM, "lib"), f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}", "-lrocprofiler-sdk-roctx"])
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
