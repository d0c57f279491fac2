"""Builds libnbody.so (HIP, gfx950) in-tree with hipcc.

``python -m paper_2303_12166_amd.build`` or ``build()`` from Python. Packed FP32 instructions are
switched off for the whole library (``-packed-fp32-ops``), so every FP32 operation is a plain
VOP2/VOP3 instruction.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libnbody.so")
SOURCES = [os.path.join(CSRC, "nb_kernels.hip"), os.path.join(CSRC, "nb_probe.hip"),
           os.path.join(CSRC, "nb_runtime.cpp")]
ARCH = "gfx950"

HIP_FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libnbody)")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *HIP_FLAGS, "-shared", "-I", INCLUDE, "-I", CSRC, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("libnbody build failed")
    os.replace(tmp, LIB)
    return LIB


def emit_asm(out_path: str) -> str:
    """Writes the gfx950 assembly of the kernels (for inspection)."""
    cmd = [hipcc(), *HIP_FLAGS, "--cuda-device-only", "-S", "-I", INCLUDE, "-I", CSRC, "-o",
           out_path, SOURCES[0]]
    subprocess.run(cmd, check=True)
    return out_path


if __name__ == "__main__":
    print(build(verbose=True))
