"""Compile the C oracle (``amber_oracle.c``) to ``liboracle.so`` with gcc.

Building the checker is not using it; ``__graft_entry__.build()`` calls this.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "amber_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


SANITIZE = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
            "-fno-omit-frame-pointer"]


def build(verbose: bool = False, sanitize: bool = False, out: str = None) -> str:
    """liboracle.so; with sanitize, an AddressSanitizer + UndefinedBehavior
    Sanitizer build (load it with gcc's libasan preloaded) at `out`."""
    lib = out or (os.path.join(HERE, "liboracle_asan.so") if sanitize else LIB)
    # -ffp-contract=off: no float expression is fused beyond what the source
    # writes (fmaf is called where a fused multiply-add is meant)
    cmd = ["gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", "-fPIC", "-shared", "-ffp-contract=off",
           *(SANITIZE if sanitize else []), SRC, "-o", lib + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
