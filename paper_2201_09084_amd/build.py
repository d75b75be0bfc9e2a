"""Builds libpmlpic.so (HIP, gfx950) in-tree with hipcc.

Every translation unit is compiled for gfx950 only, with packed-FP32 instruction
selection disabled and hardware float atomics enabled, then linked into one shared
library next to this file.  build(check=True) builds the bounds-checked debug library
libpmlpic_check.so (-DPMLPIC_CHECK: the particle kernels check their indices before each
access and the host reports failed checks as errors); binding.py loads it when the
environment variable PMLPIC_LIB names it.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpmlpic.so")
LIB_CHECK = os.path.join(HERE, "libpmlpic_check.so")
SOURCES = ["api.hip", "fields.hip", "particles.hip", "push3d.hip", "fused3d.hip", "diag.hip", "batch.hip", "adjoint.hip",
           "adjoint_particles.hip", "beam.hip", "probe.hip"]

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
COMMON = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def build(verbose: bool = False, check: bool = False) -> str:
    objdir = os.path.join(ROOT, "_build", "pmlpic_check" if check else "pmlpic")
    os.makedirs(objdir, exist_ok=True)
    lib = LIB_CHECK if check else LIB
    extra = ["-DPMLPIC_CHECK"] if check else []

    def compile_one(src):
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [HIPCC] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
