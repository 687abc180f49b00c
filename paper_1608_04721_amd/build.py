"""Build libpbf.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

The library lands next to this file; the Python binding loads it from
there.  Packed FP32 instructions are switched off for device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB = PKG / "libpbf.so"
SOURCES = [CSRC / "pbf_kernels.hip", CSRC / "pbf_adjoint.hip", CSRC / "pbf_api.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and Path(cand).exists():
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libpbf)")


def compile_cmd(out: Path, extra=()):
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-I", str(ROOT / "include"),
            *map(str, SOURCES), "-o", str(out), *extra]


def build(verbose: bool = False) -> Path:
    """Compile every source into libpbf.so (always recompiles)."""
    tmp = LIB.with_suffix(".so.tmp")
    cmd = compile_cmd(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed to build libpbf.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
