"""Build the oracle's shared library (test infrastructure) with the host C
compiler: plain C99, -O2, no fast-math and no floating-point contraction, so
each rounding in oracle.c is exactly the one written there."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, source: str = None, out: str = None) -> str:
    source = source or os.path.join(HERE, "oracle.c")
    out = out or LIB
    cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-frounding-math", "-Wall", "-Wextra", "-I", HERE,
           source, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
