"""Build the gfx950 HIP library ``libeqs.so`` in-tree with hipcc.

Every source under ``csrc/`` is compiled for gfx950 only; packed-FP32
instruction selection is switched off for device code.

``build_sanitized()`` builds the test driver ``tests/native/bin/abi_sanitize``:
the same sources and the driver, with AddressSanitizer and
UndefinedBehaviorSanitizer on the host code only (every sanitizer flag is
passed through ``-Xarch_host``; the device code is built as above).
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(ROOT, "_build", "libeqs")
LIB = os.path.join(HERE, "libeqs.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ROCM_LIB = "/opt/rocm/lib"  # roctx ranges (rocprofiler-sdk-roctx)
ARCH = "gfx950"

SOURCES = ["api.cpp", "setup.cpp", "solver.cpp", "profile.cpp", "kernels.hip", "mlp.hip", "guess.hip", "batch.cpp"]

COMMON = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # keep kernel-argument loads in the entry block: sunk into the branches that use them, they are issued and
    # waited for one batch at a time before a kernel's first data load
    "-mllvm", "-disable-machine-sink",
    "-Wall",
    "-Wno-unused-function",
    "-I", INCLUDE,
    "-I", CSRC,
]


SAN_OBJDIR = os.path.join(ROOT, "_build", "sanitize")
SAN_DRIVER = os.path.join(ROOT, "tests", "native", "abi_sanitize.cpp")
SAN_EXE = os.path.join(ROOT, "tests", "native", "bin", "abi_sanitize")
# host code only: each flag reaches the host compilation and the link, not the device code
# (_GLIBCXX_ASSERTIONS adds libstdc++'s bounds checks of vector and string indexing)
SAN_FLAGS = [f for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
                            "-fno-omit-frame-pointer", "-g", "-D_GLIBCXX_ASSERTIONS")
             for f in ("-Xarch_host", flag)]


def _compile(src: str, objdir: str = OBJDIR, extra=()) -> str:
    obj = os.path.join(objdir, os.path.basename(src) + ".o")
    path = src if os.path.isabs(src) else os.path.join(CSRC, src)
    cmd = [HIPCC, *COMMON, *extra, "-x", "hip", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int = 4) -> str:
    """Compile all sources and link ``libeqs.so``; returns the library path."""
    os.makedirs(OBJDIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-L", ROCM_LIB, "-Wl,-rpath," + ROCM_LIB,
           "-lrocprofiler-sdk-roctx"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def build_sanitized(jobs: int = 4) -> str:
    """Compile the library's sources and the sanitizer driver with host-side
    ASan/UBSan and link the driver executable; returns its path."""
    os.makedirs(SAN_OBJDIR, exist_ok=True)
    os.makedirs(os.path.dirname(SAN_EXE), exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, SAN_OBJDIR, SAN_FLAGS), [*SOURCES, SAN_DRIVER]))
    tmp = SAN_EXE + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", *SAN_FLAGS, "-o", tmp, *objs, "-L", ROCM_LIB,
           "-Wl,-rpath," + ROCM_LIB, "-lrocprofiler-sdk-roctx"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, SAN_EXE)
    return SAN_EXE


if __name__ == "__main__":
    jobs = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    print(build(jobs))
    if "--sanitize" in sys.argv[2:]:
        print(build_sanitized(jobs))
