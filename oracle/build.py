"""Build the FP64 CPU oracle (plain C, gcc) into oracle/liboracle.so.

Test infrastructure: the oracle is only loaded by the test suite, the smoke check and the
benchmark's CPU-baseline leg."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["quad.c", "geodesic.c", "tables.c", "emission.c", "render.c", "animate.c", "march.c", "bloom.c", "tonemap.c", "area.c", "spectrum.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-Wno-unused-parameter", "-o", LIB + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES]
    cmd += ["-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
