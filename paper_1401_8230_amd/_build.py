"""Build libprngd.so in-tree with hipcc for gfx950."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libprngd.so")
OBJ_DIR = os.path.join(HERE, "_build")

# One translation unit per kernel family, compiled in parallel.  The family
# units are built twice: the kernels of the default Eq. (5) map, and the
# kernels that take the map's constants from the launch (FAM_ANY_MAP).
FAMILY_SOURCES = ["prngd_k_spec.hip", "prngd_k_philox.hip", "prngd_k_single.hip",
                  "prngd_k_mrg.hip", "prngd_k_ranmar.hip"]
SOURCES = ["prngd_k_triple.hip", "prngd_k_misc.hip", "prngd_noalloc.hip", "prngd_probes.hip",
           "prngd_runtime.cpp", "prngd_ranmar_host.cpp"]
UNITS = ([(src, "eq5", ["-DPRNGD_MAPF=0u"]) for src in FAMILY_SOURCES]
         + [(src, "anymap", ["-DPRNGD_MAPF=FAM_ANY_MAP"]) for src in FAMILY_SOURCES]
         + [(src, "", []) for src in SOURCES])
KERNEL_SOURCES = ["prngd_device.hpp", "prngd_internal.hpp", "prngd_k_misc.hip",
                  "prngd_k_triple.hip"] + FAMILY_SOURCES

# -ffp-contract=off keeps every FP64 operation of the map a separate IEEE
# operation; packed FP32 instructions are disabled for the device code.
HIPCC_FLAGS = [
    "-std=c++17", "-O3", "-fPIC", "--offload-arch=gfx950",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I" + os.path.join(ROOT, "include"),
    "-I/opt/rocm/include",
]


def kernel_source_hash():
    """First 16 hex digits of the SHA-256 of the fill kernels' sources: HBM
    counter figures are only reported for the kernels they were taken on."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return path


# Host code only (the device code is built as always): AddressSanitizer and
# UndefinedBehaviorSanitizer for the runtime, for CPU test runs with the
# clang sanitizer runtime preloaded.
SANITIZE_HOST = ["-g", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
                 "-Xarch_host", "-fsanitize=undefined"]


def _compile(unit, verbose, extra=()):
    src, tag, defines = unit
    stem = src.rsplit(".", 1)[0] + (f"_{tag}" if tag else "")
    obj = os.path.join(OBJ_DIR, stem + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else ["-x", "c++", "-D__HIP_PLATFORM_AMD__"]
    cmd = [hipcc(), *HIPCC_FLAGS, *extra, *defines, *lang, "-c", os.path.join(CSRC, src),
           "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose=False, jobs=None, sanitize_host=False):
    os.makedirs(OBJ_DIR, exist_ok=True)
    jobs = jobs or min(len(UNITS), os.cpu_count() or 1, 8)
    extra = SANITIZE_HOST if sanitize_host else []
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        objs = list(pool.map(lambda unit: _compile(unit, verbose, extra), UNITS))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
