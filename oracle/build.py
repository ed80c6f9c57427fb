"""Compile the C oracle into oracle/liboracle.so (test infrastructure only).

The sampling decisions are pinned binary32 arithmetic, so the file is built
without floating-point contraction and without fast-math.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["oracle.c", "shade.c", "neural.c", "dct.c"]
TARGET = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, src_dir: str = HERE, target: str = TARGET) -> str:
    """Compile the oracle's C sources found in src_dir into target (the
    defaults build oracle/liboracle.so; the tests build planted-mistake
    copies elsewhere)."""
    srcs = [os.path.join(src_dir, s) for s in SOURCES if os.path.exists(os.path.join(src_dir, s))]
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
           "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", target + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(target + ".tmp", target)
    return target


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
