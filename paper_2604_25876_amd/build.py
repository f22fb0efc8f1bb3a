"""Build the HIP library libskyr.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
SOURCES = [PKG / "csrc" / "skyr.hip"]
DEPS = SOURCES + [PKG / "csrc" / n for n in ("sweep.hpp", "shapes.hpp", "moments.hpp", "formp.hpp")] + \
    [ROOT / "include" / "skyr.h"]
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


def build_sanitized(out: Path, verbose: bool = False) -> Path:
    """The library with AddressSanitizer and UndefinedBehaviorSanitizer in its host code,
    for runs of the CPU tests over the host runtime (argument checks, planning, files,
    host-side draws); nothing in such a run launches a kernel.  The device code is built
    without sanitizers and with one tile shape per precision, which keeps the build short.
    Load it with SKYR_LIB=<out> and the clang ASan runtime preloaded."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out = Path(out)
    tmp = out.with_suffix(".so.tmp")
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-fno-omit-frame-pointer",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-fvisibility=hidden",
           "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined",
           "-DSKYR_SHAPES_F64(X)=X(4, 4, 1, 16, 1, 1.0)", "-DSKYR_SHAPES_F32(X)=X(8, 4, 1, 32, 1, 1.0)",
           "-I", str(ROOT / "include"), "-o", str(tmp), *map(str, SOURCES)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def asan_runtime() -> str:
    """The clang AddressSanitizer runtime that a SKYR_LIB sanitizer build needs preloaded."""
    root = Path(os.environ.get("ROCM_PATH", "/opt/rocm")) / "llvm" / "lib" / "clang"
    found = sorted(root.glob("*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        raise FileNotFoundError(f"no libclang_rt.asan-x86_64.so under {root}")
    return str(found[-1])


def stale() -> bool:
    return not LIB.exists() or any(d.stat().st_mtime > LIB.stat().st_mtime for d in DEPS)


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
