"""Build step of the test-only unit-kernel library (tests/csrc/libppc_unit.so):
the library's device header compiled into small kernels that the GPU unit
tests drive."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
LIB = os.path.join(HERE, "libppc_unit.so")


def build() -> str:
    from paper_2412_16370_amd import build as hipbuild

    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipbuild.hipcc(), "--offload-arch=" + hipbuild.ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2412_16370_amd", "csrc"),
           "-o", tmp, os.path.join(HERE, "unit_kernels.hip")]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        noise = "is not a recognized feature for this target"
        raise RuntimeError("hipcc failed:\n" + "\n".join(l for l in proc.stderr.splitlines() if noise not in l))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
