"""Compile the C oracle (``amber_oracle.c``) to ``liboracle.so`` with gcc.

Building the checker is not using it; ``__graft_entry__.build()`` calls this.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "amber_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    # -ffp-contract=off: no float expression is fused beyond what the source
    # writes (fmaf is called where a fused multiply-add is meant)
    cmd = ["gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", "-fPIC", "-shared", "-ffp-contract=off",
           SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
