"""Builds paper_2211_15963_amd/libdbsim.so for gfx950 with hipcc (host cross-compiles; no GPU needed).

Flags that matter for results: -ffp-contract=off (no fused multiply-add, so each
float operation rounds once), no fast-math, f32 denormals preserved, and packed
FP32 instructions disabled.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build", "dbsim")
ARCH = os.environ.get("DBSIM_OFFLOAD_ARCH", "gfx950")

HIPFLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
            "-fno-gpu-flush-denormals-to-zero", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
            "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
SOURCES = ["kernels.hip", "devbuild.hip", "netbuild.cpp", "abi.cpp"]


def hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("compile failed: " + " ".join(cmd[-3:]))
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    jobs = []
    objs = []
    for s in SOURCES:
        o = os.path.join(BUILD, os.path.splitext(s)[0] + ".o")
        objs.append(o)
        jobs.append([cc, "-x", "hip", *HIPFLAGS, "-c", os.path.join(CSRC, s), "-o", o])
    o = os.path.join(BUILD, "dbnet.o")
    objs.append(o)
    jobs.append(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-I",
                 os.path.join(ROOT, "include"), "-c", os.path.join(ROOT, "netgen", "dbnet.c"), "-o", o])
    with ThreadPoolExecutor(max_workers=4) as ex:
        list(ex.map(lambda c: _run(c, verbose), jobs))
    out = os.path.join(HERE, "libdbsim.so")
    _run([cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", out + ".tmp", "-lpthread", "-lm"], verbose)
    os.replace(out + ".tmp", out)
    return out


def asm(source: str = "kernels.hip") -> str:
    """Device assembly of one source (for inspecting our own gfx950 code)."""
    os.makedirs(BUILD, exist_ok=True)
    o = os.path.join(BUILD, os.path.splitext(source)[0] + f"-{ARCH}.s")
    _run([hipcc(), "-x", "hip", *HIPFLAGS, "--cuda-device-only", "-S", os.path.join(CSRC, source), "-o", o], False)
    return o


if __name__ == "__main__":
    print(build(verbose=True))
