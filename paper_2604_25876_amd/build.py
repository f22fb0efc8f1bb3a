"""Build the HIP library libskyr.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
SOURCES = [PKG / "csrc" / "skyr.hip"]
DEPS = SOURCES + [PKG / "csrc" / "sweep.hpp", PKG / "csrc" / "moments.hpp", PKG / "csrc" / "formp.hpp", ROOT / "include" / "skyr.h"]
LIB = PKG / "libskyr.so"

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wall",
]


def build(verbose: bool = False, extra: list[str] | None = None) -> Path:
    """Compile libskyr.so (always recompiles)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [hipcc, *HIPCC_FLAGS, *(extra or []), "-I", str(ROOT / "include"), "-o", str(tmp), *map(str, SOURCES)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    return not LIB.exists() or any(d.stat().st_mtime > LIB.stat().st_mtime for d in DEPS)


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
