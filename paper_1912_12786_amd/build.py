"""Builds librtx.so (HIP, gfx950 only) in-tree with hipcc.

Run as ``python -m paper_1912_12786_amd.build``.  The library is written next
to this file so that it travels with the source tree.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB_PATH = os.path.join(HERE, "librtx.so")
SOURCES = ["rtx_capi.cpp", "bvh_build.cpp", "trace_kernels.hip", "hit_backward.hip",
           "bvh_refit.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # bit-reproducible float32: no contraction, IEEE division, no flushing
    "-ffp-contract=off",
    "-fno-fast-math",
    "-fno-gpu-flush-denormals-to-zero",
    # never emit packed fp32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build librtx)")


def build(verbose: bool = False) -> str:
    """Compiles every source into ``librtx.so``; always rebuilds."""
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    cc = hipcc()
    for src in SOURCES:
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        cmd = [cc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-x", "hip", "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        # the host pass does not know the gfx950-only packed-fp32 feature: harmless
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                        if "packed-fp32-ops' is not a recognized feature" not in l)
        if msg.strip():
            print(msg, file=sys.stderr)
        if r.returncode != 0:
            raise subprocess.CalledProcessError(r.returncode, cmd)
        objs.append(obj)
    tmp = LIB_PATH + ".tmp"
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def build_user_library(sources, out_path: str, verbose: bool = False) -> str:
    """Compiles HIP sources that instantiate the traversal template with their
    own intersector (they include ``csrc/rt_launch.hpp``) into a shared
    library at ``out_path``, with the same flags as librtx."""
    cc = hipcc()
    objs = []
    for src in sources:
        obj = os.path.splitext(out_path)[0] + "_" + os.path.splitext(os.path.basename(src))[0] + ".o"
        cmd = [cc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-x", "hip", "-c", src,
               "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                        if "packed-fp32-ops' is not a recognized feature" not in l)
        if msg.strip():
            print(msg, file=sys.stderr)
        if r.returncode != 0:
            raise subprocess.CalledProcessError(r.returncode, cmd)
        objs.append(obj)
    tmp = out_path + ".tmp"
    subprocess.run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], check=True)
    os.replace(tmp, out_path)
    for o in objs:
        os.remove(o)
    return out_path


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv[1:]))
