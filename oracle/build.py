"""Build the FP64 oracle shared library (test infrastructure only).

The oracle is compiled with plain gcc, IEEE semantics (no fast-math, no FMA
contraction).  The step code is compiled twice: once in double and once in
double complex (complex-step derivatives).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD, "libvbd_oracle.so")

CFLAGS = ["-O2", "-fPIC", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    units = [("oracle_core.c", "core_r.o", ["-DOR_COMPLEX=0"]),
             ("oracle_core.c", "core_c.o", ["-DOR_COMPLEX=1"]),
             ("oracle_prep.c", "prep.o", [])]
    for src, obj, extra in units:
        out = os.path.join(BUILD, obj)
        cmd = ["gcc", *CFLAGS, *extra, "-c", os.path.join(HERE, src), "-o", out]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        objs.append(out)
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-shared", "-fopenmp", "-o", tmp, *objs, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
