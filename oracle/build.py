"""Compile oracle.cpp into liboracle.so next to this file (plain g++, strict IEEE: no fast-math and no
FMA contraction, so every operation rounds as written), and the same source with OpenMP into
liboracle_omp.so (the all-threads timing variant of the Krylov kernels; the parity tests use the
serial library)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
OUT = os.path.join(HERE, "liboracle.so")
OUT_OMP = os.path.join(HERE, "liboracle_omp.so")
# -O3 without -march=native: the library built here also runs on the GPU host, whose CPU may lack
# instructions this one has; strict IEEE either way (no fast-math, no contraction, so no reordering)
FLAGS = ["-std=c++17", "-O3", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-Wextra",
         "-Wno-unused-parameter", "-Wno-unknown-pragmas"]
FLAGS_SHOWN = ["-O3", "-fno-fast-math", "-ffp-contract=off", "(-fopenmp for the all-threads build)"]


def build(verbose=False):
    for out, extra in ((OUT, []), (OUT_OMP, ["-fopenmp"])):
        cmd = ["g++", *FLAGS, *extra, SRC, "-o", out + ".tmp"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return OUT


def compiler_version():
    r = subprocess.run(["g++", "--version"], capture_output=True, text=True)
    return r.stdout.splitlines()[0] if r.returncode == 0 and r.stdout else "g++"


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
