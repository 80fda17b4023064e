"""Compiles the oracle's plain C helpers (test infrastructure) with gcc.

Each ``oracle/csrc/*.c`` becomes ``oracle/_<name>.so``; the oracle loads them
with ctypes. Nothing here is linked into, or loaded by, the GPU library.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")


def lib_path(name: str) -> str:
    return os.path.join(HERE, f"_{name}.so")


def build(verbose: bool = False) -> list[str]:
    out = []
    if not os.path.isdir(CSRC):
        return out
    for f in sorted(os.listdir(CSRC)):
        if not f.endswith(".c"):
            continue
        name = f[:-2]
        dst = lib_path(name)
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-o", dst + ".tmp",
               os.path.join(CSRC, f), "-lm"]
        p = subprocess.run(cmd, capture_output=True, text=True)
        if p.returncode != 0:
            raise RuntimeError(f"oracle C build failed: {' '.join(cmd)}\n{p.stderr}")
        os.replace(dst + ".tmp", dst)
        out.append(dst)
        if verbose:
            print(f"built {dst}")
    return out


if __name__ == "__main__":
    build(verbose=True)
