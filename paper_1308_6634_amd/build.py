"""Build the HIP library ``libplsqr.so`` in-tree for gfx950.

Kernels are compiled by hipcc for gfx950 only; the host engine is plain C++ compiled
by the ROCm clang; the shared object is linked by hipcc. Usage:
``python -m paper_1308_6634_amd.build`` (or ``build()`` from Python).
"""

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libplsqr.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

KERNEL_SOURCES = ["kernels.hip", "smooth_vec.hip", "blur.hip", "dense.hip", "gemm_bf16.hip",
                  "ring.hip", "static_scratch.hip", "zmarch.hip",
                  "tail_lds.hip"]
HOST_SOURCES = ["driver.cpp", "api.cpp"]
HEADERS = ["plsqr_internal.hpp", "kernels.hpp", "engine.hpp", "device_common.hpp", "finalize.hpp"]

# Packed-FP32 instructions are disabled for every device compile (the compiler would
# otherwise form v_pk_* FP32 ops from ordinary float code). Kernel arguments are preloaded
# into SGPRs at wave launch (gfx950), so a kernel's first descriptor load does not wait for a
# load of its own arguments; the code object keeps a prologue that loads them from memory when
# the firmware does not preload.
DEVICE_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
                "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics", "-mllvm",
                "-amdgpu-kernarg-preload-count=16", "-Wall", "-Wno-unused-result"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__", "-Wall", "-Wno-unused-value"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=True):
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    clang = os.path.join(ROCM, "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = shutil.which("g++")
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", os.path.join(ROCM, "include")]
    jobs = []
    for src in KERNEL_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append((obj, [hipcc, "-c", *DEVICE_FLAGS, *inc, os.path.join(CSRC, src), "-o", obj]))
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append((obj, [clang, "-x", "c++", "-c", *HOST_FLAGS, *inc, os.path.join(CSRC, src),
                           "-o", obj]))
    # the translation units are independent: compile them side by side
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", "8"))))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        for fut in [ex.submit(_run, cmd, verbose) for _, cmd in jobs]:
            fut.result()
    objs = [obj for obj, _ in jobs]
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp,
          "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lpthread"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
