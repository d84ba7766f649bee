"""Build the CPU oracle library (test infrastructure only).

gcc, -O2, no FMA contraction, no fast-math, SSE2 doubles: every FP64
operation in the oracle is one IEEE round-to-nearest-even operation.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liboracle.so")

CFLAGS = ["-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
          "-fno-fast-math", "-msse2", "-mfpmath=sse", "-Wall", "-Wextra"]


# AddressSanitizer and UndefinedBehaviorSanitizer, for CPU test runs with
# gcc's sanitizer runtimes preloaded.
SANITIZE = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=undefined"]


def build(verbose=False, sanitize=False):
    os.makedirs(OUT_DIR, exist_ok=True)
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, *(SANITIZE if sanitize else []), "-o", tmp,
           os.path.join(HERE, "prngd_oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
