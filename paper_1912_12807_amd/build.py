"""Build libfdas.so in-tree with hipcc for gfx950.

Every HIP source is compiled with packed FP32 instructions disabled (the
compiler is not allowed to fuse FP32 pairs into v_pk_* forms), host sources
with the same compiler in C++ mode. The result lands next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfdas.so")

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function"]
HOST_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    hip = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    cpp = sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp"))
    return hip, cpp


def _compile(src: str, flags, obj: str):
    cmd = [hipcc()] + flags + ["-I", CSRC, "-I", INCLUDE, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r.stderr


def build(verbose: bool = False, out: str = None, obj_dir: str = None, defines=()) -> str:
    """Compile and link; out/obj_dir/defines let tuning builds go elsewhere."""
    lib = out or LIB
    obj = obj_dir or OBJ
    os.makedirs(obj, exist_ok=True)
    extra = [f"-D{d}" for d in defines]
    hip, cpp = sources()
    jobs = []
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        for f in hip:
            jobs.append(ex.submit(_compile, f, HIP_FLAGS + extra, os.path.join(obj, f + ".o")))
        for f in cpp:
            jobs.append(ex.submit(_compile, f, ["-x", "c++"] + HOST_FLAGS + extra, os.path.join(obj, f + ".o")))
        for j in jobs:
            err = j.result()
            if verbose and err:
                print(err, file=sys.stderr)
    objs = [os.path.join(obj, f + ".o") for f in hip + cpp]
    tmp = lib + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
