"""Build the oracle's shared library with gcc (test infrastructure only)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libckks_oracle.so")


def build(force: bool = True) -> str:
    """Compile oracle/ckks_oracle.c into oracle/libckks_oracle.so and return its path."""
    if not force and os.path.exists(LIB):
        return LIB
    src = os.path.join(HERE, "ckks_oracle.c")
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
                           "-shared", "-fPIC", "-o", tmp, src, "-lm"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
