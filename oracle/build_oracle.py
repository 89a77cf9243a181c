"""Build the oracle shared library (plain C, single-threaded).

Test infrastructure only: compiled by ``__graft_entry__.build()`` and by the
test-suite when the library is missing.  ``-ffp-contract=off`` keeps every
IEEE double operation of the Poisson threshold rule separately rounded.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mclg_oracle.c")
LIB = os.path.join(HERE, "libmclg_oracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off",
           "-fno-fast-math", "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build())
