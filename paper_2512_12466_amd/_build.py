"""Build libnyxrt.so for gfx950 with hipcc (cross-compiles without a GPU).

FP contraction is off so that every decision quantity is a single correctly
rounded operation; packed FP32 instructions are disabled; FP atomics compile
to the hardware instructions.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libnyxrt.so")
SOURCES = ["capi.hip", "trace.hip", "spectrum.hip", "chem.hip", "merge.hip", "noalloc.hip"]
ARCH = os.environ.get("NYXRT_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(verbose: bool = False, extra=()) -> str:
    cmd = [HIPCC] + FLAGS + ["-I" + INCLUDE] + list(extra) + sources() + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=CSRC)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
