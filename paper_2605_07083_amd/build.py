"""Build the gfx950 HIP library ``libpic.so`` in-tree with hipcc."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpic.so")
SOURCES = ["pic_kernels.hip", "pic_host.hip", "surrogate_kernels.hip", "surrogate_host.hip"]
ARCH = os.environ.get("PIC_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags():
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function"]


def build(verbose=False):
    out = LIB + ".tmp"
    cmd = [hipcc()] + flags() + ["-shared", "-o", out] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(out, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
