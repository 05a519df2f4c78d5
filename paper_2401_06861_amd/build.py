"""Build the HIP engine for gfx950 into paper_2401_06861_amd/libnwq.so.

    python -m paper_2401_06861_amd.build      (or __graft_entry__.build())

Every .hip file under csrc/ is compiled to an object in csrc/_build/ with
hipcc (in parallel), then linked into one shared library exporting the C ABI
of include/nwq.h.  Packed FP32 instructions are disabled for device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(CSRC, "_build")
LIB = os.path.join(PKG, "libnwq.so")
ARCH = os.environ.get("NWQ_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


# The register-blocked SV kernel holds 16 amplitudes per thread in arrays
# indexed by compile-time constants and alternates two such register sets
# between gates.  Sinking the stores common to the cases of its gate switch
# into the join block (an early LLVM CFG simplification) leaves a run-time
# index, and the arrays then live in scratch memory; it is turned off for that
# file.
FILE_FLAGS = {
    "kernels_fuse.hip": ["-mllvm", "-simplifycfg-sink-common=false"],
}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, *FILE_FLAGS.get(os.path.basename(src), []), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources for {ARCH}", file=sys.stderr)
    return LIB


# Host-side checking build: every source with AddressSanitizer and
# UndefinedBehaviorSanitizer on its host code only (the device code is built
# as usual, without them), linked against the shared sanitizer runtime.  The
# library then serves the device-free entry points (argument validation, the
# OpenQASM reader, the fusion planner) in a CPU process that preloads that
# runtime; it is not used on a GPU.
SAN_DIR = os.path.join(BUILD, "san")
SAN_LIB = os.path.join(SAN_DIR, "libnwq_san.so")
SAN_FLAGS = [f"--offload-arch={ARCH}", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Wno-unused-command-line-argument"]


def sanitizer_runtime() -> str:
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return r.stdout.strip()


def build_sanitized(verbose: bool = True) -> str:
    os.makedirs(SAN_DIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))

    def one(src):
        obj = os.path.join(SAN_DIR, os.path.basename(src) + ".o")
        r = subprocess.run([HIPCC, *SAN_FLAGS, *FILE_FLAGS.get(os.path.basename(src), []), "-c", src, "-o", obj],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc (host, sanitizers) failed on {src}:\n{r.stdout}\n{r.stderr}")
        return obj

    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(one, srcs))
    r = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-shared-libsan",
                        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                        "-o", SAN_LIB, *objs], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link (sanitizers) failed:\n{r.stdout}\n{r.stderr}")
    if verbose:
        print(f"built {SAN_LIB} (ASan and UBSan on host code)", file=sys.stderr)
    return SAN_LIB


if __name__ == "__main__":
    if sys.argv[1:] == ["sanitized"]:
        build_sanitized()
    else:
        build()
