"""Builds the C oracle (test infrastructure) into oracle/liboracle.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRCS = [os.path.join(HERE, "oracle.c")]
FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-Wall", "-shared", "-fPIC"]


# the stand-alone driver the sanitizer test builds with AddressSanitizer and
# UndefinedBehaviorSanitizer; build() only checks that it compiles
DRIVER = os.path.join(HERE, "sanitize_driver.c")


def build(force=True):
    if not force and os.path.exists(LIB) and all(
            os.path.getmtime(LIB) >= os.path.getmtime(s) for s in SRCS + [os.path.join(HERE, "oracle.h")]):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", *FLAGS, "-o", tmp, *SRCS, "-lm"])
    os.replace(tmp, LIB)
    subprocess.check_call(["gcc", "-fsyntax-only", "-Wall", "-Wno-unknown-pragmas", DRIVER])
    return LIB


if __name__ == "__main__":
    print(build())
