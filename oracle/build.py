"""Build the CPU oracle shared library (test infrastructure) with gcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["mech.c", "chem.c", "rodas.c", "mapping.c", "mlp.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    # Portable x86-64-v3 code (AVX2/FMA) so the library built here also runs on
    # the GPU host; no floating-point contraction, so the mixture fraction is
    # evaluated with separately rounded multiplies and adds.
    cmd = ["gcc", "-std=gnu11", "-O3", "-march=x86-64-v3", "-ffp-contract=off",
           "-fno-math-errno", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           "-o", LIB + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
