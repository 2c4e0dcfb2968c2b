"""Compile the HIP library for gfx950 (in-tree, one hipcc invocation)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", "fss_lib.hip"), os.path.join(HERE, "csrc", "shuffle.hip"),
        os.path.join(HERE, "csrc", "access.hip")]
SRC = SRCS[0]
HEADERS = [os.path.join(HERE, "csrc", "aes_gfx950.hpp"), os.path.join(HERE, "csrc", "chacha_gfx950.hpp"),
           os.path.join(HERE, "csrc", "common.hpp"),
           os.path.join(ROOT, "include", "oblivgm_fss.h")]
LIB = os.path.join(HERE, "liboblivgm_fss.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-function",
    # packed-FP32 instructions stay off in every HIP build of this project
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    """Always recompiles (the caller asked for a build)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *HIPCC_FLAGS, "-o", tmp, *SRCS]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(ln for ln in res.stdout.splitlines() if "packed-fp32-ops" not in ln and "hip-link" not in ln)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    if verbose and out.strip():
        print(out)
    os.replace(tmp, LIB)
    return LIB


def needs_build() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in [*SRCS, *HEADERS])


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
