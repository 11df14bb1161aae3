"""Build the gfx950 HIP library liblbkt.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblbkt.so")
SOURCES = [os.path.join(HERE, "csrc", n) for n in ("lbkt.hip", "vn.hip", "noalloc.hip")]
DEPS = SOURCES + [os.path.join(HERE, "csrc", "kt_site.hpp"), os.path.join(HERE, "csrc", "lbkt_internal.hpp"),
                  os.path.join(ROOT, "include", "lbkt.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # every fused multiply-add is explicit in the source; nothing else is contracted
    "-ffp-contract=off",
    # no packed FP32 instructions in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False) -> str:
    """Compile liblbkt.so (always recompiles); returns its path."""
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I" + os.path.join(ROOT, "include"), "-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
