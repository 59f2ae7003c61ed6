"""Build libcrb.so (HIP, gfx950) in-tree.

Steps: regenerate the median networks (csrc/gen_networks.py -> csrc/medtile.inc),
compile each HIP translation unit with hipcc for gfx950, link the shared library
next to this file.  Floating-point flags: no contraction into FMA (the binary64
statistics follow the plain definition's operation order), no NaN handling in
min/max (inputs are finite by contract), packed FP32 arithmetic disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "libcrb.so")
SOURCES = ["detect.hip", "kernels.hip", "farm.hip", "api.hip", "server.hip"]
ARCH = os.environ.get("CRB_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
          "-fno-honor-nans", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    return out


def generate_networks() -> None:
    sys.path.insert(0, CSRC)
    try:
        import gen_networks
        gen_networks.generate(os.path.join(CSRC, "medtile.inc"))
    finally:
        sys.path.pop(0)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    generate_networks()

    def compile_one(src):
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        out = _run([HIPCC] + CFLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
        if verbose and out.strip():
            print(out)
        return obj

    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
