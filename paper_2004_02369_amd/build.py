"""Build libpg.so (HIP for gfx950 + host C++) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpg.so")
ROWBENCH = os.path.join(HERE, "librowbench.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SOURCES = ["api.cpp", "plan.cpp", "ingest.cpp", "engine.hip"]
HEADERS = ["pg_internal.hpp", "engine.hpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", f"-I{INCLUDE}"]
# Device code: gfx950 only; packed fp32 instructions disabled (this code has no
# fp32 math, the flag keeps the compiler from emitting them anywhere).
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    def compile_one(src):
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        return obj, _run([HIPCC, *COMMON, *DEVICE, *lang, "-c", path, "-o", obj])

    # the sources compile independently: one hipcc per source, side by side
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        results = list(ex.map(compile_one, SOURCES))
    objs = []
    for obj, out in results:
        if verbose and out:
            print(out)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, *DEVICE, "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    # the measurement kernels (streaming reads, row-pair intersections)
    tmp = ROWBENCH + ".tmp%d" % os.getpid()
    _run([HIPCC, *COMMON, *DEVICE, "-x", "hip", "-shared", os.path.join(CSRC, "rowbench.hip"), "-o", tmp])
    os.replace(tmp, ROWBENCH)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
