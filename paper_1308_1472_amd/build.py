"""Builds libfcx.so (HIP for gfx950 + host C++) in-tree with hipcc.

    python -m paper_1308_1472_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libfcx.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# packed FP32 instructions are kept out of the device code on purpose
DEVICE_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
                "-Wno-unused-variable", "-Wno-unused-but-set-variable"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall"]

HOST_SOURCES = ["forest.cpp"]
DEVICE_SOURCES = ["api.hip"]


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    jobs = []
    for src in HOST_SOURCES:
        obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
        jobs.append(["g++", *HOST_FLAGS, *inc, "-c", os.path.join(CSRC, src),
                     "-o", obj])
        objs.append(obj)
    for src in DEVICE_SOURCES:
        obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
        jobs.append([HIPCC, *DEVICE_FLAGS, *inc, "-c", os.path.join(CSRC, src),
                     "-o", obj])
        objs.append(obj)
    procs = [subprocess.Popen(j, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
             for j in jobs]
    failed = False
    for j, p in zip(jobs, procs):
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the device target feature
        text = "\n".join(l for l in text.splitlines()
                         if "packed-fp32-ops' is not a recognized" not in l)
        if p.returncode != 0 or (verbose and text.strip()):
            print(" ".join(j), file=sys.stderr)
            print(text, file=sys.stderr)
        failed |= p.returncode != 0
    if failed:
        raise RuntimeError("libfcx build failed")
    tmp = LIB + ".tmp"
    subprocess.run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp,
                    *objs], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
