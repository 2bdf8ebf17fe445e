"""Compiles the plain-C oracle (test infrastructure) with gcc into oracle/libkz_oracle.so."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "kz_oracle.c"), os.path.join(HERE, "kz_oracle_ext.c")]
LIB = os.path.join(HERE, "libkz_oracle.so")


def build_oracle(force: bool = False) -> str:
    """Builds the oracle library if it is missing or older than its source; returns its path."""
    if (not force and os.path.exists(LIB)
            and all(os.path.getmtime(LIB) >= os.path.getmtime(f) for f in SRCS)):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", tmp] + SRCS
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_oracle(force=True))
