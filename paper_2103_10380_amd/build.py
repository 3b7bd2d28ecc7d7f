"""Builds libfastnerf.so (the render library: all its HIP sources, gfx950) and
liblinebench.so (the line-gather measurement kernels used by bench.py) in the
package directory."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libfastnerf.so")
SOURCES = ["fastnerf_kernels.hip", "fastnerf_api.hip", "fastnerf_serve.hip", "fastnerf_bake.hip",
           "fastnerf_direction.hip"]
LINEBENCH_SRC = "linebench.hip"
LINEBENCH_LIB = os.path.join(PKG, "liblinebench.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
         # no packed FP32 instructions: some of their forms have been unreliable here
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _compile(src: str, obj: str, verbose: bool):
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")


def build(verbose: bool = False) -> str:
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objs = [os.path.join(objdir, s.replace(".hip", ".o")) for s in srcs]
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        list(ex.map(lambda p: _compile(p[0], p[1], verbose), zip(srcs, objs)))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    lb_obj = os.path.join(objdir, LINEBENCH_SRC.replace(".hip", ".o"))
    _compile(LINEBENCH_SRC, lb_obj, verbose)
    tmp = LINEBENCH_LIB + ".tmp"
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, lb_obj],
                   check=True)
    os.replace(tmp, LINEBENCH_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
