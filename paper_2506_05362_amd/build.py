"""Compile the HIP sources of the package into in-tree shared libraries for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")

# Packed FP32 instructions stay disabled; FP64 work never needs them anyway.
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"]

LIBS = {
    "libpd_mi355x.so": ["pd_kernels.hip", "pd_api.hip"],
    "libpd_mlp.so": ["mlp.hip"],
}
# roctx ranges around the host-side phases of a step (shown by rocprofv3 --marker-trace)
LINK = {
    "libpd_mi355x.so": ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx"],
}


def build(verbose: bool = False) -> list:
    out = []
    for lib, srcs in LIBS.items():
        target = os.path.join(PKG, lib)
        tmp = target + ".tmp"
        cmd = ["hipcc", *HIPFLAGS, *[os.path.join(CSRC, s) for s in srcs], *LINK.get(lib, []), "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, target)
        out.append(target)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
