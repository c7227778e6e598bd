"""Build of the HIP library (gfx950) into paper_2202_01284_amd/libdrt.so."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdrt.so")
SOURCES = ["drt_kernels.hip", "drt_nrc.hip", "drt_wavefront.hip", "drt_host.cpp"]
# per-source extra flags: the kernels use the hardware's approximate (about
# 1 ulp) float division and square root instead of correctly rounded
# sequences, and flush float32 denormals (values below 2^-126 play no part in
# the renderer's arithmetic), so a reciprocal or square root is one
# instruction instead of a range-scaled sequence of five or six
KERNEL_FLAGS = ["-fno-hip-fp32-correctly-rounded-divide-sqrt", "-fgpu-flush-denormals-to-zero"]
EXTRA = {"drt_kernels.hip": KERNEL_FLAGS, "drt_nrc.hip": KERNEL_FLAGS,
         "drt_wavefront.hip": KERNEL_FLAGS}
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-munsafe-fp-atomics",
    # no packed FP32 instructions (v_pk_*_f32): some of their forms have given
    # wrong results on this hardware; the FP32 VALU peak counts them out
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    """Compile every source for gfx950 and link libdrt.so (always rebuilds)."""
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *FLAGS, *EXTRA.get(src, []), "-x", "hip", "-c", os.path.join(CSRC, src),
               "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
