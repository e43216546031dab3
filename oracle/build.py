"""Build the oracle's shared library with gcc (test infrastructure only).

The oracle is plain C compiled with -O2, OpenMP over independent blocks, and
no FMA contraction, so its arithmetic is the IEEE double arithmetic written in
the source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "librlt2_oracle.so")
SOURCES = [os.path.join(HERE, "rlt2_oracle.c")]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           "-o", LIB + ".tmp"] + SOURCES + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def needs_build() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = SOURCES + [os.path.join(HERE, "rlt2_oracle.h")]
    return any(os.path.getmtime(s) > t for s in deps)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
