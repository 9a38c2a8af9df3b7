"""Compile the C oracle into ``libmsm_oracle.so`` next to its sources."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["msm_oracle.c", "md_oracle.c"]
LIB = os.path.join(HERE, "libmsm_oracle.so")


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = SOURCES + ["msm_oracle.h", "md_oracle.h"]
    return any(os.path.getmtime(os.path.join(HERE, s)) > t
               for s in deps if os.path.exists(os.path.join(HERE, s)))


def compile_oracle(force: bool = True) -> str:
    if not force and not stale():
        return LIB
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-Wno-unused-parameter", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(compile_oracle())
