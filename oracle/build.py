"""Build the C oracle into oracle/liblb_oracle.so (plain gcc, OpenMP).

Test infrastructure only: the product library never links or loads it.

Flags: -O3 with -ffp-contract=off, so that no multiply-add is fused and every
operation rounds as written (the checker's arithmetic stays the plain FP64
definition, independent of the host's instruction set).  The portable build
(the tests' checker) targets generic x86-64; the CPU-baseline timing builds a
second copy with -march=native on the host that times it, which gives the
same results bit for bit (no contraction, no reassociation) at the host's best
vector width.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lb_oracle.c")
LIB = os.path.join(HERE, "liblb_oracle.so")
LIB_NATIVE = os.path.join(HERE, "liblb_oracle_native.so")

FLAGS = ["-O3", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall"]


def build(force: bool = False, native: bool = False) -> str:
    lib = LIB_NATIVE if native else LIB
    if not force and os.path.exists(lib) and os.path.getmtime(lib) >= os.path.getmtime(SRC):
        return lib
    cmd = ["gcc"] + FLAGS + (["-march=native"] if native else []) + ["-o", lib + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    print(build(force="--force" in sys.argv, native="--native" in sys.argv))
