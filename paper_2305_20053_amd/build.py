"""Build the C-ABI shared library libsaa.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsaa.so")
SOURCES = ["api.cpp", "model.cpp", "train.cpp", "linalg.cpp", "ouu.cpp", "pde_all.hip", "cvar.hip", "mlp.hip", "train.hip",
           "eig.hip", "gemm.hip", "tune.cpp"]
ARCH = os.environ.get("SAA_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False) -> str:
    """Compile every source for gfx950 and link libsaa.so; returns its path."""
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    flags = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             # packed FP32 instructions are kept out of all device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
    cmds = []
    for src in SOURCES:
        obj = os.path.join(bdir, src + ".o")
        cmds.append((src, [hipcc()] + flags + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]))
        objs.append(obj)

    def compile_one(item):
        src, cmd = item
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, stderr=None if verbose else subprocess.PIPE, text=True)
        return src, res.returncode, res.stderr or ""

    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1)), 16))
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        for src, rc, err in ex.map(compile_one, cmds):
            if rc != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lrocblas"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
