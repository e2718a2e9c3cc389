"""Build step for the oracle's shared library (test infrastructure only).

Compiles ``shgo_oracle.cpp`` with the host compiler into ``liboracle.so`` next to this file.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "shgo_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")


def build(force=True):
    """Compile the oracle. With ``force=False`` an existing, up-to-date library is kept."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["g++", "-O2", "-std=gnu++17", "-fopenmp", "-fPIC", "-shared", SRC, "-o", tmp, "-lquadmath"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
