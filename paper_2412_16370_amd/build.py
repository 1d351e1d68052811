"""Build step of the HIP library: compiles every ``csrc/*.hip`` for gfx950
into ``libppc.so`` next to this file (in-tree, so it travels with the
source tree)."""
from __future__ import annotations

import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libppc.so")
ARCH = os.environ.get("PPC_OFFLOAD_ARCH", "gfx950")


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def command(out: str) -> list[str]:
    return [
        hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
        # packed fp32 VALU forms stay off (none of this code is fp32, but
        # the flag keeps the compiler from ever emitting them)
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function",
        "-I" + os.path.join(ROOT, "include"),
        "-I" + os.path.join(HERE, "csrc"),
        "-o", out,
    ] + sources() + ["-lpthread"]


def build() -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    proc = subprocess.run(command(tmp), capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(ln for ln in proc.stderr.splitlines() if noise not in ln)
    if proc.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
