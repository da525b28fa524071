"""Build step for the CPU oracle (test infrastructure): gcc -> libsps_oracle.so."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sps_oracle.c")
LIB_PATH = os.path.join(HERE, "libsps_oracle.so")


def build(src: str = SRC, out: str = LIB_PATH) -> str:
    """Compile the oracle (always recompiles).  Returns the library path."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
