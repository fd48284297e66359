"""Build the CPU oracle (plain C, gcc + OpenMP) into oracle/liboracle*.so.

Test infrastructure: the oracle is only loaded by the test suite, the smoke
check and the CPU-baseline leg of the benchmark.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_LD = os.path.join(HERE, "liboracle_ld.so")


def build(force: bool = True) -> None:
    """Compile the FP64 oracle and its long-double twin."""
    for out, extra in ((LIB, []), (LIB_LD, ["-DORACLE_LONG_DOUBLE"])):
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
            continue
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-Wno-unused-function", *extra, "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)


if __name__ == "__main__":
    build()
