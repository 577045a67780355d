"""Compile the C oracle into oracle/libdsg_oracle.so (host gcc; test
infrastructure only)."""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

HERE = Path(__file__).resolve().parent
LIB = HERE / "libdsg_oracle.so"


def build() -> Path:
    tmp = LIB.with_suffix(".so.tmp")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           str(HERE / "peel_oracle.c"), str(HERE / "cbds_oracle.c"), "-o", str(tmp)]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise RuntimeError("oracle build failed: " + " ".join(cmd))
    os.replace(tmp, LIB)
    return LIB


def ensure() -> Path:
    if not LIB.exists():
        build()
    return LIB


if __name__ == "__main__":
    print(build())
