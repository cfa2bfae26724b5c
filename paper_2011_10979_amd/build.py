"""Build libflowmi.so (HIP kernels + C ABI runtime) for gfx950 with hipcc, in-tree, and the plain C
client of its C ABI (tests/c_client/solve_pair) with gcc.

Usage: python -m paper_2011_10979_amd.build [--jobs N]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libflowmi.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SOURCES = ["admm.hip", "admm_tb.hip", "admm_rows.hip", "pyramid.hip", "pdr.hip", "pdr_tb.hip", "pdr_rows.hip", "alg1_tb.hip", "alg1_rows.hip", "energy.hip", "noalloc.hip",
           "runtime.cpp", "geometry.cpp", "context.cpp", "tb_plan.cpp", "autotune.cpp", "batch.cpp", "multi.cpp", "serve.cpp"]

ARCH = os.environ.get("FLOWMI_ARCH", "gfx950")
C_CLIENT_SRC = os.path.join(os.path.dirname(HERE), "tests", "c_client", "solve_pair.c")
C_CLIENT = os.path.splitext(C_CLIENT_SRC)[0]


def hipcc() -> str:
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm install expected under /opt/rocm)")


def common_flags():
    return ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
            # packed FP32 instructions are disabled: the compiler would otherwise emit them itself
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-Wno-unused-variable"]


def compile_one(src: str) -> str:
    os.makedirs(BUILD, exist_ok=True)
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc()] + common_flags() + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int = 8, verbose: bool = False) -> str:
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    build_c_client(verbose)
    return LIB


def build_c_client(verbose: bool = False) -> str:
    """Compile the C client as C11 with gcc against include/flow.h, libflowmi.so and the HIP runtime
    (found at run time through an rpath relative to the binary, so the tree can move)."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        raise RuntimeError("no C compiler (gcc) found")
    tmp = C_CLIENT + ".tmp"
    cmd = [cc, "-std=c11", "-O2", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"),
           "-I", INCLUDE, C_CLIENT_SRC, "-o", tmp, "-L", HERE, "-lflowmi", "-L", os.path.join(rocm, "lib"),
           "-lamdhip64", "-lm", "-Wl,-rpath,$ORIGIN/" + os.path.relpath(HERE, os.path.dirname(C_CLIENT)), f"-Wl,-rpath,{os.path.join(rocm, 'lib')}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"C client build failed\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, C_CLIENT)
    if verbose:
        print(f"built {C_CLIENT}")
    return C_CLIENT


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    a = ap.parse_args(argv)
    build(a.jobs, verbose=True)


if __name__ == "__main__":
    sys.exit(main())
