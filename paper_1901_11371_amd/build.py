"""Compile the hbf shared library (host construction + HIP kernels for gfx950)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
OUT = os.path.join(OUT_DIR, "libhbf.so")

HOST_SOURCES = ["hankel.cpp", "plan.cpp", "schedule.cpp", "ctx.cpp", "solver.cpp"]
DEVICE_SOURCES = ["stage.hip", "stage_pipe.hip", "stage_mfma.hip", "stage_lanes.hip", "gmres.hip", "noalloc.hip",
                  "entries.hip"]

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-fcx-limited-range",
             # packed FP32 instructions stay disabled (see the build notes)
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(line for line in r.stdout.splitlines() if "packed-fp32-ops" not in line)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    objs = []
    obj_dir = os.path.join(OUT_DIR, "obj")
    os.makedirs(obj_dir, exist_ok=True)
    from concurrent.futures import ThreadPoolExecutor

    def one(src):
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            return None
        obj = os.path.join(obj_dir, src + ".o")
        cmd = ["hipcc"] + HIP_FLAGS + ["-c", path, "-o", obj]
        if src.endswith(".cpp"):
            cmd = ["hipcc", "-O3", "-std=c++17", "-fPIC", "-fcx-limited-range", "-march=x86-64-v3", "-c", path,
                   "-o", obj]
        _run(cmd)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        for o in ex.map(one, HOST_SOURCES + DEVICE_SOURCES):
            if o:
                objs.append(o)
    tmp = OUT + ".tmp"
    _run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"])
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
