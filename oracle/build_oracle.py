"""Compile the FP64 CPU oracle (test infrastructure) into oracle/libsrot_oracle.so.

Plain gcc, no FMA contraction, so every double operation in the oracle is the
separately rounded IEEE operation written in its source.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "srot_oracle.c")
LIB = os.path.join(HERE, "libsrot_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
