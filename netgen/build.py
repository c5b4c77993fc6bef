"""Builds netgen/libdbnet.so (the seeded network generator) with gcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    out = os.path.join(HERE, "libdbnet.so")
    cmd = ["gcc", *CFLAGS, "-shared", "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "dbnet.c"),
           "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
