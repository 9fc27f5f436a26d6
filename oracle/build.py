"""Build the oracle's shared library (test infrastructure only).

The oracle is plain C99 compiled with gcc -O2 and no fast-math or FP
contraction, so every FP64 operation is a single correctly rounded IEEE
operation.  Run ``python -m oracle.build`` or call :func:`build`.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["healpix.c", "spectrum.c", "trace.c", "merge.c", "chem.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c99", "-D_GNU_SOURCE", "-O2", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
           "-pthread", "-o", LIB + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


SANITIZERS = {"address": "address,undefined", "thread": "thread"}


def build_sanitized(kind: str, out: str) -> str:
    """The oracle with sanitize_main.c as a host executable built with gcc
    under AddressSanitizer + UndefinedBehaviorSanitizer ("address") or
    ThreadSanitizer ("thread")."""
    cmd = ["gcc", "-std=c99", "-D_GNU_SOURCE", "-O1", "-g", "-fno-omit-frame-pointer",
           "-ffp-contract=off", "-fno-fast-math", f"-fsanitize={SANITIZERS[kind]}",
           "-fno-sanitize-recover=all", "-pthread", "-I" + HERE, "-o", out]
    cmd += [os.path.join(HERE, s) for s in SOURCES + ["sanitize_main.c"]] + ["-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
