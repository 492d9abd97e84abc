"""Build the FP64 CPU oracle (test infrastructure) with gcc into oracle/liblbpf_oracle.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "lbpf_oracle.c"), os.path.join(HERE, "sp_oracle.c"),
        os.path.join(HERE, "d3q15_oracle.c")]
LIB = os.path.join(HERE, "liblbpf_oracle.so")


def build(verbose=False):
    # -O2 keeps strict IEEE double semantics: no -ffast-math, no FMA contraction, so that
    # the oracle evaluates every formula in the order it is written.
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
           "-o", LIB + ".tmp"] + SRCS + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
