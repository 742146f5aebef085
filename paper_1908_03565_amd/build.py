"""Builds libjxlr.so, the HIP library of the package, for gfx950.

hipcc compiles the kernels and the C-ABI host code into
paper_1908_03565_amd/libjxlr.so.  Packed-FP32 instructions are disabled for
the device code; they are not needed and have been unreliable here.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libjxlr.so")
SOURCES = [os.path.join(CSRC, f) for f in ("jxlr_kernels.hip", "jxlr_tables.cpp")]
ARCH = os.environ.get("JXLR_OFFLOAD_ARCH", "gfx950")


def build(verbose: bool = False) -> str:
    sys.path.insert(0, CSRC)
    import gen_dct_consts
    gen_dct_consts.generate()
    cmd = ["/opt/rocm/bin/hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
           "-shared", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-result",
           *SOURCES, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
