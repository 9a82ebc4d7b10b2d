"""Compile the FP64 CPU oracle into oracle/libst_oracle.so with gcc.

Test infrastructure: only the tests, the smoke check and the benchmark's
CPU-baseline leg load the result.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "st_oracle.c")
PAR = os.path.join(HERE, "st_oracle_par.c")
LIB = os.path.join(HERE, "libst_oracle.so")

# -ffp-contract=off: every multiply and add is rounded as written.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-Wall"]


def build(src=SRC, out=LIB, extra=()):
    """The serial oracle plus its particle-parallel drivers (OpenMP)."""
    cmd = ["gcc", *CFLAGS, "-fopenmp", *extra, src, PAR, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build(*sys.argv[1:2]) if len(sys.argv) > 1 else build())
