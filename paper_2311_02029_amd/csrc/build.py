"""Builds libmetatrinity.so for gfx950 with hipcc (one object per source)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
OUT = os.path.join(PKG, "libmetatrinity.so")
SOURCES = ["runtime.hip", "seq.hip", "index.hip", "classify.hip", "filter.hip", "fused.hip", "server.hip", "tune.hip", "contain.hip",
           "abundance.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


TORCH_ALLOC_OUT = os.path.join(PKG, "libmt_torch_alloc.so")


def build_torch_alloc(out: str = TORCH_ALLOC_OUT, verbose: bool = False) -> str:
    """The binding's shim that hands PyTorch's caching allocator to
    mt_set_allocator (host C++ against the installed torch)."""
    import torch
    tdir = os.path.dirname(torch.__file__)
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__", "-DUSE_ROCM",
           "-I", os.path.join(tdir, "include"), "-I", "/opt/rocm/include", os.path.join(HERE, "torch_alloc.cpp"),
           "-L", os.path.join(tdir, "lib"), "-lc10_hip", "-lc10", "-Wl,-rpath," + os.path.join(tdir, "lib"),
           "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"torch allocator shim failed:\n{r.stdout}\n{r.stderr}")
    os.replace(out + ".tmp", out)
    return out


def build(out: str = OUT, verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = ["hipcc", *FLAGS, "-c", os.path.join(HERE, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = out + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    build_torch_alloc(verbose=verbose)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
