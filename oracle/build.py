"""Compile the serial CPU oracle (test infrastructure) into oracle/_build/liboracle.so.

Only tests, the smoke check and the benchmark's CPU-baseline leg load the
result; the GPU library never does.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpm_oracle.c")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liboracle.so")


def build(sanitize: bool = False, out: str = LIB) -> str:
    os.makedirs(os.path.dirname(out), exist_ok=True)
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-shared", "-fPIC", SRC, "-o", out, "-lm"]
    if sanitize:
        cmd[3:3] = ["-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    subprocess.run(cmd, check=True)
    return out


def ensure_built() -> str:
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    return LIB


if __name__ == "__main__":
    print(build(sanitize="--sanitize" in sys.argv))
