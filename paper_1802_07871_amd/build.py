"""Compile the HIP library (libctbop.so) for gfx950, in place."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libctbop.so")
SOURCES = ["ctbop.hip", "ctbop_dev.h", "k_lists.h", "k_tersoff.h", "k_qeq.h", "k_md.h", "server.h", "dual.h",
           "k_adjoint.h", "adjoint_host.h", "removal.h", "k_rings.h", "rings_host.h", "static_entry.h", "k_fq.h"]


def hipcc_cmd(out: str) -> list[str]:
    return ["hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            # packed FP32 instructions stay off in every kernel
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Werror=uninitialized", "-Wno-unused-function", "-Wno-unused-variable",
            os.path.join(CSRC, "ctbop.hip"), "-o", out]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = hipcc_cmd(tmp)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to build libctbop.so")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
