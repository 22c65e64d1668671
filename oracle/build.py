"""Compile the CPU oracle (test infrastructure) into ``oracle/liborc.so``."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "skiplist.c")
LIB = os.path.join(HERE, "liborc.so")


SELFTEST = os.path.join(HERE, "selftest.c")
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def build_selftest(out: str, sanitize: bool = True) -> str:
    """The oracle's self-test driver (selftest.c) as an executable, built with
    AddressSanitizer and UndefinedBehaviorSanitizer (host code only)."""
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-Wall", "-Wextra", *(SANITIZE if sanitize else []), SRC, SELFTEST,
           "-o", out]
    subprocess.run(cmd, check=True)
    return out


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", SRC, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
