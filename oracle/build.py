"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

The oracle is plain C compiled by gcc with floating-point contraction off, so
every product and sum is rounded separately as the source reads.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["lsd_oracle.c", "mpnn_oracle.c", "pair_oracle.c", "net_oracle.c"]
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wno-unused-function", "-Wno-maybe-uninitialized", "-o", OUT + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
