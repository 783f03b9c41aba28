"""Compile the CPU oracle (test infrastructure) into oracle/liboracle.so.

The oracle is plain C99 built with gcc; it is used only by tests, the smoke
check and the benchmark's CPU-baseline leg.  The same source is also built
with OpenMP into oracle/liboracle_omp.so, a timing mode for the CPU baseline
only (the sequential library is the one every check uses).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")
SRC = os.path.join(HERE, "oracle.c")
CFLAGS = ["-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unknown-pragmas"]


def _compile(out, extra, verbose, src=SRC):
    tmp = out + ".tmp"
    cmd = ["gcc", *CFLAGS, *extra, "-fPIC", "-shared", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    _compile(LIB, [], verbose)
    _compile(LIB_OMP, ["-fopenmp"], verbose)
    return LIB


def build_variant(src: str, out: str, verbose: bool = False) -> str:
    """Build a sequential oracle library from another source file (the
    mutation tests compile deliberately altered copies this way)."""
    return _compile(out, ["-I" + HERE, "-w"], verbose, src=src)


if __name__ == "__main__":
    print(build(verbose=True))
