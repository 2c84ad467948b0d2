"""Compile the oracle (plain C, FP64) into ``oracle/liboracle.so``.

Test infrastructure only.  ``-ffp-contract=off`` and no fast-math keep every
product and sum an individually rounded IEEE-754 double operation.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# The Cholesky oracle is a library of its own (its mutation tests rebuild it
# alone).
CHOL_SRC = os.path.join(HERE, "cholesky.c")
CHOL_LIB = os.path.join(HERE, "liboracle_chol.so")
# The tiled LU oracle likewise.
LU_SRC = os.path.join(HERE, "lu.c")
LU_LIB = os.path.join(HERE, "liboracle_lu.so")


def _compile(src, lib):
    tmp = lib + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)


def build(force: bool = True) -> str:
    for src, lib in ((SRC, LIB), (CHOL_SRC, CHOL_LIB), (LU_SRC, LU_LIB)):
        if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
            _compile(src, lib)
    return LIB


if __name__ == "__main__":
    print(build())
