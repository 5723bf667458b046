"""Build the gfx950 shared library libgmf.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgmf.so")
SOURCES = ["gmf_kernels.hip", "gmf_sample.hip", "gmf_mstep.hip", "gmf_fft.hip", "gmf_runtime.cpp"]
ARCH = os.environ.get("GMF_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are kept out of the generated code on purpose.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel, one hipcc per file) and link libgmf.so."""
    jobs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = ["hipcc", *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((src, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    objs, failed = [], []
    for src, obj, proc in jobs:
        _, stderr = proc.communicate()
        # the host pass does not know the packed-fp32 feature; that warning is harmless
        err = "\n".join(l for l in stderr.splitlines() if "packed-fp32-ops" not in l)
        if proc.returncode != 0:
            failed.append(f"hipcc failed for {src}:\n{err}")
        elif err.strip() and verbose:
            print(err, file=sys.stderr)
        objs.append(obj)
    if failed:
        raise RuntimeError("\n".join(failed))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
