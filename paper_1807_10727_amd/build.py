"""Compile the HIP library libcc.so for gfx950 (in-tree, next to this file)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcc.so")
SOURCES = ["lc_kernels.hip", "lc_sort.hip", "lc_bucket.hip", "lc_fused.hip", "lc_tiled.hip", "lc_variants.hip",
           "lc_engine.hip", "lc_batch.hip", "lc_serve.hip"]
ARCH = os.environ.get("PYTORCH_ROCM_ARCH", "gfx950")


def command(out: str = LIB):
    return (["hipcc", "--offload-arch=%s" % ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
             # no packed fp32 instructions in any kernel
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument", "-pthread",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", out]
            + [os.path.join(CSRC, s) for s in SOURCES])


def build() -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    proc = subprocess.run(command(tmp), stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout)
        raise RuntimeError("hipcc failed building libcc.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
