"""Build libmgrit.so (HIP kernels + host driver) in-tree for gfx950.

Each source is compiled to an object in its own process (in parallel), then
the objects are linked into the shared library.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libmgrit.so")
CSRC = os.path.join(PKG, "csrc")
SOURCES = [os.path.join(CSRC, f) for f in ("mgrit_step_poly_z.hip", "mgrit_step_poly_w.hip", "mgrit_step_slc.hip",
                                           "mgrit_step32_poly_z.hip", "mgrit_step32_poly_w.hip", "mgrit_step32_slc.hip",
                                           "mgrit_lean.hip", "mgrit_window.hip", "mgrit_window32.hip", "mgrit_noalloc.hip", "mgrit_gmres.hip",
                                           "mgrit_tile4.hip", "mgrit_tile8.hip", "mgrit_tile16.hip",
                                           "mgrit_kernels.hip", "mgrit_2d.hip", "mgrit_host.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
BUILD_DIR = os.path.join(PKG, "_build")


def compile_flags(arch="gfx950"):
    return [
        f"--offload-arch={arch}", "-O3", "-std=c++17", "-fPIC",
        # no packed FP32 instructions in generated code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-result",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    ]


def object_path(src):
    return os.path.join(BUILD_DIR, os.path.basename(src) + ".o")


def compile_command(src, arch="gfx950"):
    return [HIPCC, *compile_flags(arch), "-c", "-o", object_path(src), src]


def link_command(out=LIB, arch="gfx950"):
    return [HIPCC, f"--offload-arch={arch}", "-shared", "-fPIC", "-o", out, *[object_path(s) for s in SOURCES]]


def build_command(out=LIB, arch="gfx950"):
    """One-line equivalent of the build (all sources in one hipcc call)."""
    return [HIPCC, *compile_flags(arch), "-shared", "-o", out, *SOURCES]


def build_library(verbose=False):
    """Compile every HIP source into paper_2209_06916_amd/libmgrit.so."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    cmds = [compile_command(s) for s in SOURCES]
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        results = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
    failed = False
    for c, r in zip(cmds, results):
        if r.stdout:
            sys.stdout.write(r.stdout)
        err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
        if err:
            sys.stderr.write(err + "\n")
        if r.returncode != 0:
            failed = True
            sys.stderr.write(f"failed: {' '.join(c)}\n")
    if failed:
        raise subprocess.CalledProcessError(1, "hipcc")
    tmp = LIB + ".tmp"
    link = link_command(tmp)
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build_library(verbose=True)
