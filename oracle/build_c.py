"""Compile the oracle's C helper (oracle/_ctrace.so) with gcc.  Oracle code."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ctrace.c")
LIB = os.path.join(HERE, "_ctrace.so")


def build():
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", SRC, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
