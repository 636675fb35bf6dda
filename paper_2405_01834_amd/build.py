"""Builds libmderi.so (all HIP sources under csrc/) for gfx950 with hipcc.

Objects go to ``_build/`` next to this file; the shared library is written
in-tree as ``libmderi.so`` so that it travels with the source tree.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmderi.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", CSRC,
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(line for line in (r.stderr or "").splitlines() if noise not in line)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    return obj, err


def build(verbose: bool = False) -> str:
    """Compiles every source and links libmderi.so; returns its path."""
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    objs = []
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        for obj, err in ex.map(_compile, srcs):
            objs.append(obj)
            if verbose and err.strip():
                print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    # rocSOLVER / rocBLAS: the Cholesky solve of the density-fitting metric
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-L/opt/rocm/lib", "-lrocsolver",
           "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


HOSTSAN = os.path.join(HERE, "hostsan")
CLANGXX = "/opt/rocm/llvm/bin/clang++"


def build_hostsan(verbose: bool = False) -> str:
    """The host-sanitizer variant: host.hip (all host logic of the library:
    validation, pair selection, plans, workspace) compiled with
    AddressSanitizer and UndefinedBehaviorSanitizer on its host side only,
    linked with the regular objects of the other sources (their host code is
    kernel launchers) into hostsan/libmderi_hostsan.so, and the ABI driver
    tests/native/abi_sanitizer.cpp built against it with both sanitizers.
    Needs the regular objects (build() first); returns the driver's path."""
    os.makedirs(HOSTSAN, exist_ok=True)
    host_src = os.path.join(CSRC, "host.hip")
    obj = os.path.join(BUILD, "host.hip.hostsan.o")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all", "-g"]
    r = subprocess.run([HIPCC, *FLAGS, *san, "-c", host_src, "-o", obj], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for the host-sanitizer object:\n" + r.stderr)
    others = [os.path.join(BUILD, os.path.basename(x) + ".o") for x in sources() if x != host_src]
    lib = os.path.join(HOSTSAN, "libmderi_hostsan.so")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", lib, obj, *others, "-L/opt/rocm/lib",
           "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("host-sanitizer link failed:\n" + r.stderr)
    exe = os.path.join(HOSTSAN, "abi_sanitizer")
    driver_flags = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    cmd = [CLANGXX, "-std=c++17", "-O1", "-g", *driver_flags, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "native", "abi_sanitizer.cpp"),
           "-o", exe, "-L", HOSTSAN, "-lmderi_hostsan", "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath,$ORIGIN", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("driver build failed:\n" + r.stderr)
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return exe


if __name__ == "__main__":
    print(build(verbose=True))
