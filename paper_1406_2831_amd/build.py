"""Build the HIP library librbicgstab.so for gfx950 (in-tree, next to this file)."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librbicgstab.so")
SOURCES = ["kernels.hip", "api.cpp", "dense.cpp"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def build(verbose: bool = False) -> str:
    """Compile every source for gfx950 and link the shared library; returns its path.

    The host-only dense algebra (small eigenproblems and factorisations of the
    recycle-space step) is compiled separately with AVX2/FMA (x86-64-v3)."""
    tmp = LIB + ".tmp"
    objs = {name: os.path.join(HERE, name.replace(".", "_") + ".o") for name in SOURCES}
    common = [hipcc(), "-O3", "-std=c++17", "-fPIC", "-pthread", "-Wno-unused-command-line-argument",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    gpu = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    steps = [
        common + ["-mavx2", "-mfma", "-c", os.path.join(CSRC, "dense.cpp"), "-o", objs["dense.cpp"]],
        common + ["-c", os.path.join(CSRC, "api.cpp"), "-o", objs["api.cpp"]],
        common + gpu + ["-c", os.path.join(CSRC, "kernels.hip"), "-o", objs["kernels.hip"]],
        common + gpu + ["-shared"] + [objs[n] for n in SOURCES] + ["-o", tmp],
    ]
    try:
        for cmd in steps:
            if verbose:
                print(" ".join(cmd), flush=True)
            res = subprocess.run(cmd, capture_output=True, text=True)
            if res.returncode != 0:
                sys.stderr.write(res.stdout + res.stderr)
                raise RuntimeError("hipcc failed building librbicgstab.so")
    finally:
        for o in objs.values():
            if os.path.exists(o):
                os.remove(o)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
