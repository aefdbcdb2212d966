"""Builds ``oracle/liboracle.so`` from ``nauticle_oracle.c`` with gcc.

Contraction of a*b+c into fused multiply-adds is disabled so that every
FP32 operation in the bit-exact part is rounded exactly as written.

``build(sanitize=True)`` builds ``oracle/liboracle_san.so`` instead, with
AddressSanitizer and UndefinedBehaviorSanitizer (host code only; any report
aborts): ``oracle/sanitize_check.py`` runs the oracle's pins against it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nauticle_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")
OUT_SAN = os.path.join(HERE, "liboracle_san.so")


def build(sanitize: bool = False) -> str:
    out = OUT_SAN if sanitize else OUT
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-pthread"]
    if sanitize:
        cmd += ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    cmd += ["-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
