"""Build the CPU oracle shared library (test infrastructure only).

    python oracle/build_oracle.py

gcc, -O2, -ffp-contract=off: no fused multiply-add, every operation rounded as
written in pcpic_oracle.c.  -fopenmp only enables the threaded orc_step_par.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pcpic_oracle.c")
LIB = os.path.join(HERE, "libpcpic_oracle.so")


def build(verbose: bool = False, src: str = SRC, out: str = LIB) -> str:
    cmd = ["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", "-Wall", "-Wextra", "-I", HERE, "-o", out, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, capture_output=not verbose)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
