"""Compile the FP64 CPU oracle into ``oracle/liboracle.so`` (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark load
the result.  Plain gcc, no GPU toolchain involved.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pic_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def _compile(out, extra):
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
           "-D_GNU_SOURCE"] + extra + ["-o", out + ".tmp", SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


def build(force: bool = True) -> str:
    """The single-threaded oracle (liboracle.so) and the same source built with
    OpenMP over its per-particle loops (liboracle_omp.so), whose results are
    identical: the threads share only integer sums and the order-dependent
    work stays in particle order."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    _compile(LIB, [])
    _compile(LIB_OMP, ["-fopenmp"])
    return LIB


if __name__ == "__main__":
    print(build())
