"""Build ``libtitan.so`` (HIP, gfx950) in-tree.

Every translation unit under ``csrc/`` is compiled with hipcc for gfx950 in
parallel, then linked into ``paper_1911_10274_amd/libtitan.so``.  Packed FP32
instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libtitan.so")
BUILD_DIR = os.path.join(ROOT, "_build", "titan")

ARCH = "gfx950"
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", f"--offload-arch={ARCH}",
          "-I", INCLUDE, "-I", CSRC]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libtitan)")


def sources() -> list[str]:
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def build(verbose: bool = False, defines: dict | None = None, out: str | None = None) -> str:
    """Compile and link.  ``defines`` adds -D macros (e.g. the tiled kernel's
    TITAN_TILE / TITAN_UNROLL / TITAN_NT_LOADS tuning knobs) and ``out`` puts
    the library elsewhere; the defaults build the shipped library."""
    defines = defines or {}
    tag = "_".join(f"{k}{v}" for k, v in sorted(defines.items()))
    bdir = os.path.join(BUILD_DIR, tag) if tag else BUILD_DIR
    os.makedirs(bdir, exist_ok=True)
    out = out or LIB
    cc = hipcc()
    srcs = sources()
    dflags = [f"-D{k}={v}" for k, v in sorted(defines.items())]

    def compile_one(src):
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        cmd = [cc, *COMMON, *DEVICE_FLAGS, *dflags, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
