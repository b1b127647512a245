"""Compile the HIP library ``libvplbm.so`` for gfx950 (MI355X).

``python -m paper_1905_05110_amd.build`` runs hipcc on ``csrc/vplbm.hip``.  The
library is written in-tree next to this file.  Packed FP32 instructions are turned
off for device code (``-packed-fp32-ops``); hipcc's host pass warns that it does not
know the feature, which is harmless.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "vplbm.hip")
DEPS = [SRC, os.path.join(HERE, "csrc", "vplbm_device.hpp"), os.path.join(ROOT, "include", "vplbm.h")]
LIB = os.path.join(HERE, "libvplbm.so")
ARCH = os.environ.get("VPLBM_OFFLOAD_ARCH", "gfx950")

FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include")]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS)


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and not stale():
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc"] + FLAGS + ["-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd))
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for %s" % SRC)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
