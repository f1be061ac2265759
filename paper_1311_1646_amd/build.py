"""Build the HIP library libdmrg.so for gfx950 in-tree (hipcc, no JIT cache).

    python -m paper_1311_1646_amd.build [--jobs N] [--debug] [--sanitize]

--sanitize also builds libdmrg_san.so: the host C++ (planners, drivers,
channel factorization, C-ABI) compiled with AddressSanitizer and
UndefinedBehaviorSanitizer for the host only, linked with the normal device
objects.  It is loaded through DMRG_LIBRARY with the sanitizer runtime
(SANITIZER_RUNTIME below) preloaded.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libdmrg.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("DMRG_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I", os.path.join(HERE, "..", "include")]
# Packed FP32 instructions are disabled for all device code.
# Matrix-core results are kept in ordinary VGPRs (no AGPR copies of the
# accumulators around every K-chunk, and fewer registers per wave).
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics", "-mllvm", "-amdgpu-mfma-vgpr-form"]
LIBS = ["-lrocsolver", "-lrocblas"]
OUT_SAN = os.path.join(HERE, "libdmrg_san.so")
BUILD_SAN = os.path.join(HERE, "_build_san")
# host-side only: device code is never built with a sanitizer
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
       "-fsanitize=undefined"]
SANITIZER_RUNTIME = "/opt/rocm/llvm/lib/clang/22/lib/linux/libclang_rt.asan-x86_64.so"


def sources():
    out = []
    for f in sorted(os.listdir(CSRC)):
        if f.endswith(".cpp") or f.endswith(".hip"):
            out.append(os.path.join(CSRC, f))
    return out


def compile_one(src, debug):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    flags = COMMON + (["-g"] if debug else [])
    if src.endswith(".hip"):
        cmd = [HIPCC, "-x", "hip"] + DEVICE + flags + ["-c", src, "-o", obj]
    else:
        cmd = [HIPCC] + flags + ["-D__HIP_PLATFORM_AMD__", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int = 8, debug: bool = False, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: compile_one(s, debug), srcs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + \
        ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib"] + LIBS
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


def build_sanitized(jobs: int = 8, verbose: bool = False) -> str:
    """libdmrg_san.so from the host sources compiled with the sanitizers and
    the device objects of the last build() (built first if missing)."""
    dev_objs = [os.path.join(BUILD, os.path.basename(s) + ".o") for s in sources() if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in dev_objs):
        build(jobs)
    os.makedirs(BUILD_SAN, exist_ok=True)

    def one(src):
        obj = os.path.join(BUILD_SAN, os.path.basename(src) + ".o")
        flags = [f for f in COMMON if f != "-O3"] + SAN
        cmd = [HIPCC] + flags + ["-D__HIP_PLATFORM_AMD__", "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {src}\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        return obj

    host = [s for s in sources() if s.endswith(".cpp")]
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(one, host))
    tmp = OUT_SAN + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + dev_objs + \
        ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib"] + LIBS + \
        ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libasan"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT_SAN)
    if verbose:
        print(f"built {OUT_SAN}")
    return OUT_SAN


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--debug", action="store_true")
    ap.add_argument("--sanitize", action="store_true", help="also build libdmrg_san.so (host sanitizers)")
    a = ap.parse_args()
    try:
        build(a.jobs, a.debug, verbose=True)
        if a.sanitize:
            build_sanitized(a.jobs, verbose=True)
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
