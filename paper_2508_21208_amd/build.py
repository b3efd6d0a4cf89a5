"""Compile the gfx950 library `libdgswe.so` in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdgswe.so")
SOURCES = ["dgswe_api.hip", "dgswe_kernels.hip", "dgswe_p2.hip", "dgswe_ens.hip", "mesh_prep.cpp"]
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

# Packed FP32 instructions stay disabled in every HIP build of this project.
HIP_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


# Host-code sanitizers (AddressSanitizer + UndefinedBehaviorSanitizer) for a
# CPU-side check of the host preprocessing and the boundary's host code: each
# flag applies to the host compilation only (the device code is built as
# usual); the runtime is clang's shared ASan library, which the process
# loading the library must preload.
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all", "-g"]
SANITIZE_LINK = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-shared-libasan"]
LIB_SANITIZE = os.path.join(HERE, "libdgswe_asan.so")


def build(verbose: bool = True, jobs: int = 4, sanitize: bool = False) -> str:
    """Compile every source for gfx950 and link the shared library.
    sanitize=True builds `libdgswe_asan.so` (host code under ASan + UBSan)
    beside it, from objects of its own."""
    objdir = os.path.join(HERE, "_build_asan" if sanitize else "_build")
    out = LIB_SANITIZE if sanitize else LIB
    extra = SANITIZE_FLAGS if sanitize else []
    os.makedirs(objdir, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmd = [HIPCC, *HIP_FLAGS, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    rc = [p.wait() for p in procs]
    if any(rc):
        raise RuntimeError(f"hipcc failed: {rc}")
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", *(SANITIZE_LINK if sanitize else []),
           *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def asan_runtime() -> str:
    """Path of clang's shared ASan runtime that goes with the hipcc build."""
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        import glob
        cands = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        path = cands[0] if cands else ""
    return path


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
