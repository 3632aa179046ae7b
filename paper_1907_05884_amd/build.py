"""Builds libfst.so (host C++ + HIP kernels for gfx950) in-tree with hipcc.

    python -m paper_1907_05884_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libfst.so")
ARCH = os.environ.get("FST_OFFLOAD_ARCH", "gfx950")

SOURCES = ["fst_api.cpp", "fst_model.cpp", "fst_host.cpp", "fst_corrector.cpp", "fst_batched.cpp",
           "fst_kernels.hip", "fst_linalg.hip", "fst_grid.hip", "fst_mix.hip", "fst_dway.hip", "fst_mlp.hip", "fst_gram16.hip", "fst_eval_mfma.hip",
           "fst_factor_mfma.hip"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include")]
# Device code: gfx950 only; packed FP32 instructions are disabled on purpose (the compiler
# would otherwise form v_pk_* FP32 ops from scalar code).
HIPFLAGS = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Per-file device flags.  fst_linalg.hip: the one-wave diagonal-block factorisation keeps a
# 64-entry row in registers, which needs its doubly nested 64-step loops unrolled completely
# (beyond the default pragma limit).  fst_eval_mfma.hip: MFMA results in ordinary VGPRs (in
# the default accumulator registers each would cost a copy before the VALU reduction reads it).
FILE_FLAGS = {"fst_linalg.hip": ["-mllvm", "-pragma-unroll-threshold=1000000"],
              "fst_eval_mfma.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


def _compile(src: str, verbose: bool) -> str:
    os.makedirs(BUILD, exist_ok=True)
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [_hipcc(), "-x", "hip", *HIPFLAGS, *FILE_FLAGS.get(src, []), *COMMON, "-c", path, "-o", obj]
    else:
        cmd = [_hipcc(), *COMMON, "-D__HIP_PLATFORM_AMD__", "-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if verbose and warn.strip():
        print(warn, flush=True)
    return obj


def build(verbose: bool = False) -> str:
    """Compiles every source and links libfst.so next to this file; returns its path."""
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
