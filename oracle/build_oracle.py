"""Compile the oracle's C sources into shared libraries beside them.

TEST INFRASTRUCTURE ONLY.  gcc, -O2, fp-contract off and no fast-math: every
floating-point operation in the oracle is one IEEE-754 double operation.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))

FLAGS = ["-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
         "-mno-fma", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose: bool = False) -> None:
    jobs = [("wlref.c", "liboracle.so", ["-lm", "-lpthread"]),
            ("exact_tm.c", "libexact_tm.so", [])]
    for src, out, libs in jobs:
        cmd = ["gcc", *FLAGS, os.path.join(HERE, src), "-o", os.path.join(HERE, out + ".tmp"), *libs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(os.path.join(HERE, out + ".tmp"), os.path.join(HERE, out))


if __name__ == "__main__":
    build(verbose=True)
