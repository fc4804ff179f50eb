"""Build libofv.so (HIP for gfx950) in-tree with hipcc.

Each translation unit is compiled separately and in parallel, then linked
into ``paper_2509_25924_amd/libofv.so``.  Intermediate objects go to
``paper_2509_25924_amd/_build/``.
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
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libofv.so")
ARCH = os.environ.get("OFV_OFFLOAD_ARCH", "gfx950")

SOURCES = ["ofv_api.cpp", "ofv_kernels.hip", "ofv_adjoint.hip", "ofv_adj_sums.hip", "ofv_adj_scatter.hip",
           "ofv_derived.hip"] + [f"ofv_{k}_{st}_{md}.hip" for k in ("gn", "gnt")
                                                for st in ("f32", "f16", "bf16")
                                                for md in ("zero", "direct", "upsample")]

COMMON_FLAGS = [
    "-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # register arrays indexed by a wavefront-uniform index (the band kernel's
    # vertical rings, up to 5 x 25 floats) stay in registers instead of going
    # to scratch memory: the default budget for such arrays is a quarter of the
    # registers and 16 registers per array
    "-mllvm", "-amdgpu-promote-alloca-to-vector-vgpr-ratio=1",
    "-mllvm", "-amdgpu-promote-alloca-to-vector-max-regs=32",
    "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the OFV library needs the ROCm toolchain to build")


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc(), "-c", os.path.join(CSRC, src), "-o", obj] + COMMON_FLAGS
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def _stale(src: str) -> bool:
    """True when src, or any header in csrc/ or include/, is newer than its object file."""
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, src)] + [os.path.join(d, f) for d in (CSRC, INCLUDE) for f in os.listdir(d)
                                        if f.endswith(".h")]
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, jobs: int = 0, incremental: bool = False) -> str:
    """Compile every source (incremental: only sources newer than their objects, headers counted as
    dependencies of every source) and link libofv.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    todo = [s for s in SOURCES if not incremental or _stale(s)]
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda s: _compile(s, verbose), todo))
    objs = [os.path.join(BUILD, os.path.basename(s) + ".o") for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def built() -> bool:
    return os.path.exists(LIB)


if __name__ == "__main__":
    path = build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv)
    print(path)
