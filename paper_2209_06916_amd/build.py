"""Build libmgrit.so (HIP kernels + host driver) in-tree for gfx950."""
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libmgrit.so")
SOURCES = [os.path.join(PKG, "csrc", "mgrit_kernels.hip"), os.path.join(PKG, "csrc", "mgrit_host.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build_command(out=LIB, arch="gfx950"):
    return [
        HIPCC, f"--offload-arch={arch}", "-O3", "-std=c++17", "-fPIC", "-shared",
        # no packed FP32 instructions in generated code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-result",
        "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
        "-o", out, *SOURCES,
    ]


def build_library(verbose=False):
    """Compile every HIP source into paper_2209_06916_amd/libmgrit.so."""
    tmp = LIB + ".tmp"
    cmd = build_command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build_library(verbose=True)
