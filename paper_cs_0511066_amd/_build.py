"""Builds the gfx950 shared library libdet.so in-tree with hipcc.

Each source compiles to an object under paper_cs_0511066_amd/_build/, then
everything links into paper_cs_0511066_amd/libdet.so.  Used by
__graft_entry__.build() and runnable directly:  python paper_cs_0511066_amd/_build.py
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdet.so")
SOURCES = ["lu_kernels.hip", "dixon_kernels.hip", "batch_kernels.hip", "capi.cpp", "batch.cpp",
           "serve.cpp", "host_api.cpp", "noalloc.hip"]
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # packed FP32 instructions stay off (see DESIGN notes on gfx950 hazards)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # let "#pragma unroll" fully unroll the register-resident panel loops
         "-mllvm", "-pragma-unroll-threshold=1000000",
         "-Wall", "-Wno-unused-result"]


def _compile(src: str) -> str:
    obj = os.path.join(OUT, src + ".o")
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "-pthread", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
