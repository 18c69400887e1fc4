"""Build the ACR shared library (libacr.so) for gfx950 with hipcc, in-tree.

Usage: python -m paper_1701_00182_amd.build [--debug]
Every HIP source under csrc/ is compiled by hipcc, every host-only C++ source
(csrc/*.cpp: no device code) by g++, to objects in _build/ (in parallel), and
all are linked into paper_1701_00182_amd/libacr.so next to this file.
"""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libacr.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXX = os.environ.get("CXX", "g++")
ROCM_INCLUDE = "/opt/rocm/include"
HOST = ["-std=c++17", "-fPIC", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INCLUDE]

COMMON = [
    "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
    # keep the compiler from forming packed FP32 instructions (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def host_flags():
    """g++ flags of the host-only sources (also used by the sanitizer test)."""
    return HOST + ["-I", os.path.join(ROOT, "include")]


def _compile(src, opt):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if src.endswith(".cpp"):
        cmd = [CXX] + host_flags() + opt + ["-c", src, "-o", obj]
    else:
        cmd = [HIPCC] + COMMON + opt + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(debug=False, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    opt = ["-O0", "-g"] if debug else ["-O3"]
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=jobs) as pool:
        objs = list(pool.map(lambda s: _compile(s, opt), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(debug="--debug" in sys.argv, verbose=True)
