"""Build the FP64 CPU oracle (plain C, gcc) into oracle/libsu2oracle.so: the SU(2)
heat bath and, on top of its SU(2) step, the SU(3) subgroup heat bath.

Test infrastructure only: the library built here is loaded by the tests, the
smoke check and the benchmark's CPU-baseline leg, never by the product path.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, f) for f in ("su2_oracle.c", "su3_oracle.c")]
HDRS = [os.path.join(HERE, f) for f in ("su2_oracle.h", "su3_oracle.h")]
SRC = SRCS[0]
LIB = os.path.join(HERE, "libsu2oracle.so")


def stale() -> bool:
    """True when the library is missing or older than any oracle source."""
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in SRCS + HDRS)


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and not stale():
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp, *SRCS, "-lm"]
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
