"""Compile the oracle's C time loop with gcc (test infrastructure only)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle_fd.c")
LIB = os.path.join(HERE, "liboracle_fd.so")


def build(force=True):
    """Build liboracle_fd.so next to its source. IEEE FP64, no fast-math."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O3", "-fPIC", "-shared", "-std=c99",
                           "-fno-fast-math", "-ffp-contract=off", "-o", tmp, SRC])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
