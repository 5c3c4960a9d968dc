"""Builds libpamc.so (HIP for gfx950) in the package directory.

Every translation unit is compiled by hipcc with FP contraction off (the
weight normalisation must round exactly like the host code) and without
packed-FP32 instructions.  Objects are compiled in parallel and linked into
one shared library with a plain C ABI (include/pamc.h).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpamc.so")
SOURCES = ["sweep.hip", "gather.hip", "resample.hip", "icm.hip", "calib.hip", "static_run.hip", "runner.cpp",
           "pamc_api.cpp", "server.cpp", "tune.cpp", "instances.cpp"]
ARCH = os.environ.get("PAMC_OFFLOAD_ARCH", "gfx950")
ROCM_INC = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "include")


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def common_flags():
    return ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall",
            "-Wno-unused-function", "-Wno-unused-variable", "-I", os.path.join(ROOT, "include")]


def _compile(src: str, obj: str, verbose: bool):
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [hipcc(), "-x", "hip", f"--offload-arch={ARCH}", *common_flags(),
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-c", path, "-o", obj]
    else:
        cmd = [hipcc(), "-x", "c++", *common_flags(), "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INC, "-c",
               path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        futs = [ex.submit(_compile, s, os.path.join(bdir, s + ".o"), verbose) for s in SOURCES]
        for f in futs:
            objs.append(f.result())
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-ldl", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
