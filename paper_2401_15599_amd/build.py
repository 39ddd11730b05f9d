"""Build the gfx950 library libtacaw.so in-tree with hipcc (no JIT, no torch extension machinery).

    python paper_2401_15599_amd/build.py          # or __graft_entry__.build()

Every translation unit is compiled in parallel, then linked into a shared library next to this
file.  Device code is built with packed-FP32 instructions disabled.  Also builds the CPU emulation
of the FFT index algebra (fft_host_check) used by the CPU test suite.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtacaw.so")
HOSTCHECK = os.path.join(HERE, "fft_host_check")
ARCH = os.environ.get("TACAW_ARCH", "gfx950")

SOURCES = ["api.cpp", "ms_kernels.hip", "pot_kernels.hip", "spec_kernels.hip", "analysis_kernels.hip"]
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I", CSRC, "-I", os.path.join(os.path.dirname(HERE), "include")]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("command failed:\n" + " ".join(cmd) + "\n" + r.stdout[-20000:])
    return r.stdout


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"]
        cmd = [HIPCC] + FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        out = _run(cmd)
        if verbose and out.strip():
            print(out)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    # CPU emulation of the FFT plans (host compiler only)
    _run(["g++", "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", CSRC,
          os.path.join(CSRC, "fft_host_check.cpp"), "-o", HOSTCHECK])
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
