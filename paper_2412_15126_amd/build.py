"""Build libckr.so (HIP kernels for gfx950 + host runtime) in-tree.

hipcc compiles the kernels and the HIP host code; g++ compiles the binary128
encoder.  Host floating point is compiled without contraction so that scale
and constant arithmetic is plain IEEE double.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libckr.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

GPU_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-function"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        sys.stderr.write(out + "\n")
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return out


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    steps = [
        ([HIPCC] + GPU_FLAGS + ["-c", os.path.join(CSRC, "ckr_kernels.hip")], "ckr_kernels.o"),
        ([HIPCC] + GPU_FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, "ckr_lib.cpp")], "ckr_lib.o"),
        (["g++", "-O2", "-std=gnu++17", "-fPIC", "-ffp-contract=off", "-Wall",
          "-c", os.path.join(CSRC, "host_math.cpp")], "host_math.o"),
    ]
    for cmd, obj in steps:
        o = os.path.join(BUILD, obj)
        out = _run(cmd + ["-o", o])
        if verbose and out:
            print(out)
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lquadmath"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
