"""Build the HIP library liblxw.so (gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblxw.so")
SOURCES = [os.path.join(CSRC, "lxw_kernels.hip"), os.path.join(CSRC, "lxw_indicator.hip"),
           os.path.join(CSRC, "lxw_host.cpp")]
HEADERS = [os.path.join(CSRC, "lxw_internal.hpp"), os.path.join(os.path.dirname(HERE), "include", "lxw.h")]

# Packed FP32 instructions are disabled for all device code (the compiler may otherwise form
# v_pk_* FP32 operations on its own).
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result"]


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc] + FLAGS + SOURCES + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
