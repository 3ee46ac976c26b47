"""Build the oracle's shared library (test infrastructure only).

The oracle is compiled with strict IEEE semantics: no fast-math and no
floating-point contraction, so every sum and product is rounded as written.
Its row loops are shared over OpenMP threads; every value is computed as in
a serial run, so the results do not depend on the thread count.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["capi.cpp"]
HEADERS = ["solver.hpp", "dual.hpp", "exact_riemann.hpp", "mlp.hpp", "cnn.hpp", "correction.hpp", "training.hpp"]
FLAGS = ["-std=c++17", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-Wall"]


def build(verbose=False):
    """Compile liboracle.so next to this file (always recompiles)."""
    cmd = ["g++"] + FLAGS + ["-o", LIB + ".tmp"] + [os.path.join(HERE, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def needs_build():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(os.path.join(HERE, f)) > t for f in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
