"""Builds the oracle's shared library with the host C compiler (no GPU code)."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    return os.path.join(_HERE, "libccmref.so")


def build_oracle() -> str:
    out = library_path()
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
           os.path.join(_HERE, "ccmref.c"), "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_oracle())
