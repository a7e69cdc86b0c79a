"""Compile the gfx950 HIP library (csrc/) into librhd.so next to this file."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = [os.path.join(HERE, "csrc", "rhd.hip"), os.path.join(HERE, "csrc", "rhd_server.hip")]
DEPS = SOURCES + [os.path.join(HERE, "csrc", f) for f in
                  ("rhd_device.hpp", "rhd_tile.hpp", "rhd_gas_tile.hpp")] + [
    os.path.join(os.path.dirname(HERE), "include", "rhd.h")]
LIB = os.path.join(HERE, "librhd.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # keep the compiler from forming packed FP32 (v_pk_*_f32) instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose=False):
    """Compile unconditionally; returns the path of the library."""
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), *HIPCC_FLAGS, "-pthread", "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def up_to_date():
    if not os.path.exists(LIB):
        return False
    t = os.path.getmtime(LIB)
    return all(os.path.getmtime(p) <= t for p in DEPS)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
