"""Builds the oracle's C part (test infrastructure only; see oracle/__init__)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tiledqr_lists.c")
LIB = os.path.join(HERE, "liboracle_lists.so")


def build_oracle(force: bool = False) -> str:
    """Compile tiledqr_lists.c with gcc into oracle/liboracle_lists.so."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_oracle(force=True))
