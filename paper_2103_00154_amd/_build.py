"""Build steps for the native parts of the package.

* ``libdsg.so``       - the HIP peeling library (gfx950) behind ``include/dsg.h``.
* ``inputs/libgraphgen.so`` - the seeded graph generators (host C, OpenMP).
* ``measure/libstream.so`` - STREAM copy / triad kernels: the measured HBM
  ceiling the benchmark reports beside the peak (gfx950).

Both are built in-tree so that the shared objects travel with the source
tree.  ``build_all()`` always recompiles; ``ensure_built()`` only builds what
is missing.
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
LIB_DSG = PKG / "libdsg.so"
LIB_GEN = PKG / "inputs" / "libgraphgen.so"
LIB_STREAM = PKG / "measure" / "libstream.so"

HIP_ARCH = "gfx950"

# Packed FP32 instructions are disabled for every HIP translation unit.
HIP_FLAGS = [
    f"--offload-arch={HIP_ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and Path(cand).exists():
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _run(cmd: list[str]) -> None:
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise RuntimeError(f"build step failed ({proc.returncode}): {' '.join(cmd)}")


def hip_sources() -> list[Path]:
    return sorted(CSRC.glob("*.hip"))


def build_dsg() -> Path:
    srcs = hip_sources()
    if not srcs:
        raise RuntimeError(f"no HIP sources under {CSRC}")
    tmp = LIB_DSG.with_suffix(".so.tmp")
    cmd = [_hipcc(), *HIP_FLAGS, f"-I{ROOT / 'include'}", *map(str, srcs), "-o", str(tmp)]
    _run(cmd)
    os.replace(tmp, LIB_DSG)
    return LIB_DSG


def build_graphgen() -> Path:
    src = PKG / "inputs" / "graphgen.c"
    tmp = LIB_GEN.with_suffix(".so.tmp")
    _run(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", str(src),
          "-lm", "-o", str(tmp)])
    os.replace(tmp, LIB_GEN)
    return LIB_GEN


def build_stream() -> Path:
    src = PKG / "measure" / "stream.hip"
    tmp = LIB_STREAM.with_suffix(".so.tmp")
    _run([_hipcc(), *HIP_FLAGS, str(src), "-o", str(tmp)])
    os.replace(tmp, LIB_STREAM)
    return LIB_STREAM


def build_all() -> None:
    build_graphgen()
    build_dsg()
    build_stream()


def ensure_graphgen() -> Path:
    if not LIB_GEN.exists():
        build_graphgen()
    return LIB_GEN


def ensure_stream() -> Path:
    if not LIB_STREAM.exists():
        build_stream()
    return LIB_STREAM


def ensure_dsg() -> Path:
    if not LIB_DSG.exists():
        build_dsg()
    return LIB_DSG
