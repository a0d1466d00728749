"""Build the HIP library liblbdem.so for gfx950 (in-tree).

    python -m paper_1711_00336_amd.build

Kernels are compiled with hipcc for gfx950 only; the host runtime and C ABI
are compiled as host C++ by the same driver and linked into one shared
library next to this file (_lib/liblbdem.so).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "liblbdem.so")
ROOT = os.path.dirname(HERE)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed FP32 VALU forms are disabled for all device code. Multiply-adds are
# fused only within one source expression (-ffp-contract=on), so a kernel
# rounds the same way whatever the surrounding code it is inlined into: the
# launch variants of one operation then agree bit for bit.
DEVICE_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-ffp-contract=on",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function"]
HOST_FLAGS = ["-O2", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        sys.stderr.write(out + "\n")
        raise RuntimeError(f"build step failed: {' '.join(cmd)}")
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    objs = []
    kern = os.path.join(CSRC, "lbdem_kernels.hip")
    ko = os.path.join(OUT_DIR, "lbdem_kernels.o")
    _run([HIPCC, *DEVICE_FLAGS, "-I", os.path.join(ROOT, "include"), "-c", kern, "-o", ko])
    objs.append(ko)
    for name in ("lbdem_capi", "lbdem_server"):
        src = os.path.join(CSRC, name + ".cpp")
        obj = os.path.join(OUT_DIR, name + ".o")
        _run([HIPCC, *HOST_FLAGS, "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj])
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
