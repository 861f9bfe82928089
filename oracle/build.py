"""Compile the CPU oracle (test infrastructure only) into oracle/liboracle.so."""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build() -> str:
    src = os.path.join(_HERE, "ref.c")
    out = os.path.join(_HERE, "liboracle.so")
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                           src, "-o", tmp, "-lm"])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
