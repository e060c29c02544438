"""Build libpolymodp.so (HIP for gfx950 only) in-tree.

    python -m paper_1402_0264_amd.build

compiles every csrc/*.hip and csrc/*.cpp with hipcc and links them into
paper_1402_0264_amd/libpolymodp.so. Packed FP32 instructions are disabled
for device code (-packed-fp32-ops); the kernels use none on purpose.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libpolymodp.so")
CALIB_SRC = os.path.join(PKG, "calib_src")
CALIB_LIB = os.path.join(PKG, "libpolymodp_calib.so")
ARCH = "gfx950"

# ROCr, for the server's SDMA copies (hsa_amd_memory_async_copy_on_engine)
LIBS = ["-L/opt/rocm/lib", "-lhsa-runtime64"]
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "--offload-arch=" + ARCH, "-I", os.path.join(ROOT, "include")]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources() -> list:
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc()] + COMMON + DEVICE_FLAGS + ["-c", "-x", "hip", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def _link(objs: list, out: str) -> None:
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-Wl,-z,defs", "-o", tmp] + objs + LIBS
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Builds libpolymodp.so and the calibration kernels (libpolymodp_calib.so)."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    calib = sorted(os.path.join(CALIB_SRC, f) for f in os.listdir(CALIB_SRC) if f.endswith(".hip"))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs) + len(calib))) as ex:
        objs = list(ex.map(_compile, srcs + calib))
    _link(objs[:len(srcs)], LIB)
    _link(objs[len(srcs):], CALIB_LIB)
    if verbose:
        print("built", LIB, "and", CALIB_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
