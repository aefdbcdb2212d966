"""Builds ``oracle/liboracle.so`` from ``nauticle_oracle.c`` with gcc.

Contraction of a*b+c into fused multiply-adds is disabled so that every
FP32 operation in the bit-exact part is rounded exactly as written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nauticle_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")


def build() -> str:
    tmp = OUT + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-pthread", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
