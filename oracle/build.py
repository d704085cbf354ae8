"""Build the CPU oracle shared libraries (test infrastructure only).

liborc64.so computes in double; liborc80.so is the same source computing in x87 long double,
used only to measure the double build's own rounding error.  Both are built with
-ffp-contract=off so that every product and sum is rounded as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dgsem_oracle.c")


def build(verbose=False):
    outs = []
    for name, extra in (("liborc64.so", []), ("liborc80.so", ["-DORC_LONG_DOUBLE"])):
        out = os.path.join(HERE, name)
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-std=c11",
               "-Wall", "-Wextra", *extra, "-o", out + ".tmp", SRC, "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
        outs.append(out)
    return outs


if __name__ == "__main__":
    for p in build(verbose=True):
        print(p)
    sys.exit(0)
