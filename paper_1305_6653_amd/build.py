"""Compile the gfx950 HIP sources into paper_1305_6653_amd/libfdebvm.so (in-tree).

    python -m paper_1305_6653_amd.build              # or __graft_entry__.build()
    python -m paper_1305_6653_amd.build --sanitize   # _build/sanitize/libfdebvm.so

The sanitizer build instruments the host code only (AddressSanitizer and
UndefinedBehaviorSanitizer through -Xarch_host; the device code is the same).  Its objects
leave the sanitizer runtime's symbols undefined: load it into a process that preloads the
runtime (``LD_PRELOAD=$(sanitizer_runtime())``) and select it with FDE_LIB_PATH.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libfdebvm.so")
SOURCES = ["k_spacetime.hip", "k_factor.hip", "k_krylov.hip", "k_gmres.hip", "k_probe.hip", "k_hessenberg.hip", "k_band.hip", "runtime.hip", "nn.hip"]
ARCH = os.environ.get("FDE_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


# roctx (named ranges for timeline tools) from the ROCm installation
LINK = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


SANITIZE_FLAGS = [
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-omit-frame-pointer",
    "-Xarch_host", "-fno-sanitize-recover=undefined",
]


def sanitizer_runtime() -> str | None:
    """Path of clang's shared AddressSanitizer runtime (it carries the UBSan handlers too)."""
    import glob
    cands = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")) + \
        sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/x86_64-unknown-linux-gnu/libclang_rt.asan.so"))
    return cands[-1] if cands else None


def _compile(src: str, outdir: str = BUILD, extra=()) -> str:
    obj = os.path.join(outdir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    outdir = os.path.join(BUILD, "sanitize") if sanitize else BUILD
    lib_path = os.path.join(outdir, "libfdebvm.so") if sanitize else LIB
    extra = SANITIZE_FLAGS if sanitize else []
    os.makedirs(outdir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, outdir, extra), SOURCES))
    tmp = lib_path + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, *LINK]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib_path)
    if verbose:
        print(f"built {lib_path}")
    return lib_path


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)
