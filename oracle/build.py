"""Compile the CPU oracle (test infrastructure) into oracle/liboracle.so."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build_from(src: str, out: str, verbose: bool = False) -> str:
    """Compile an oracle source file (oracle.c, or a copy of it) to out."""
    cmd = ["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas",
           "-I", HERE, src, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(verbose: bool = False) -> str:
    return build_from(os.path.join(HERE, "oracle.c"), LIB, verbose)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
