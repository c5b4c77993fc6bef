"""Builds oracle/liboracle.so (the CPU oracle plus the network generator) with gcc.

The oracle is test infrastructure; building it is part of the repository build so
that the checker exists, but no product code loads it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    out = os.path.join(HERE, "liboracle.so")
    cmd = ["gcc", *CFLAGS, "-shared", "-I", os.path.join(ROOT, "include"), "-I", HERE,
           os.path.join(HERE, "oracle.c"), os.path.join(ROOT, "netgen", "dbnet.c"), "-o", out + ".tmp", "-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
