"""Build the CPU oracle library (test infrastructure only).

Compiles orc_core.c twice (binary64 and binary32 modes) plus orc_grad.c (the
binary64 adjoint) and orc_math.c with
gcc into oracle/liboracle.so.  -ffp-contract=off keeps every written
operation a separately rounded IEEE-754 operation; no fast-math.
"""
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wno-unknown-pragmas"]


def build(verbose=False):
    with tempfile.TemporaryDirectory() as td:
        objs = []
        for src, defs, name in (("orc_core.c", ["-DORC_FP64"], "core64.o"),
                                ("orc_core.c", ["-DORC_FP32"], "core32.o"),
                                ("orc_grad.c", [], "grad64.o"),
                                ("orc_math.c", [], "math.o")):
            out = os.path.join(td, name)
            cmd = ["gcc", *CFLAGS, *defs, "-c", os.path.join(HERE, src), "-o", out]
            if verbose:
                print(" ".join(cmd))
            subprocess.run(cmd, check=True)
            objs.append(out)
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-shared", "-fopenmp", "-o", tmp, *objs, "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
