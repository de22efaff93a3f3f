"""Build the gfx950 shared library libotdyn.so in place with hipcc.

Every call compiles from source (no staleness check), so a build always
reflects the tree.  Sources are compiled in parallel, then linked.

`build(sanitize=True)` builds a second library, _build_asan/libotdyn_asan.so,
whose HOST code is instrumented with AddressSanitizer and
UndefinedBehaviorSanitizer (device code is compiled as usual): descriptor
validation, workspace carving, batch grouping and the other host logic.  It
is loaded by setting OT_DYN_LIB to its path and preloading the sanitizer
runtime (asan_runtime()); tests/test_sanitize.py runs the ABI tests that way.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libotdyn.so")
OBJ_ASAN = os.path.join(HERE, "_build_asan")
LIB_ASAN = os.path.join(OBJ_ASAN, "libotdyn_asan.so")
# host-only sanitizers: each -fsanitize= is for the host pass alone
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]

SOURCES = ["stencil.hip", "stencil_rows.hip", "transform.hip", "fastdct.hip", "plan.cpp",
           "batch.cpp", "otnet.hip", "net.cpp", "hue.hip", "solve_static.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-result",
]


def asan_runtime() -> str:
    """Path of the compiler's shared AddressSanitizer runtime (to preload)."""
    r = subprocess.run([os.path.join(os.path.dirname(HIPCC), "..", "llvm", "bin", "clang"),
                        "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isfile(path):
        raise RuntimeError("AddressSanitizer runtime not found")
    return path


def _compile(src: str, sanitize: bool = False) -> str:
    out = os.path.join(OBJ_ASAN if sanitize else OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *(SAN_FLAGS if sanitize else []), "-x", "hip", "-c",
           os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return out


def build(verbose: bool = False, sanitize: bool = False) -> str:
    obj, lib = (OBJ_ASAN, LIB_ASAN) if sanitize else (OBJ, LIB)
    os.makedirs(obj, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, sanitize), SOURCES))
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if sanitize:
        cmd[1:1] = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-shared-libasan"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv)
    sys.exit(0)
