"""Build the oracle's C core (test infrastructure): gcc, FP64, OpenMP.

Usage: python oracle/build.py   (writes oracle/liboracle.so)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose=False):
    src = [os.path.join(HERE, f) for f in ("sllbm_oracle.c", "sllbm_oracle_curv.c", "sllbm_oracle_mlp.c")
           if os.path.exists(os.path.join(HERE, f))]
    out = os.path.join(HERE, "liboracle.so")
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function", "-Wno-maybe-uninitialized",
           "-o", out + ".tmp"] + src + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
