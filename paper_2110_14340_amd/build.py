"""Build libjacc.so (HIP for gfx950 + the C++ runtime) in-tree.

Every source is compiled by hipcc for gfx950 only, with floating-point
contraction off (the loop bodies must round exactly like the CPU oracle),
no fast-math, and packed FP32 instructions disabled.  Objects go to
``_build/``; the shared library lands beside this file.
"""
import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libjacc.so")
ARCH = "gfx950"

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
    f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def build_id():
    """First 12 hex digits of the SHA-1 of every library source and header:
    timing databases and cost-model files are keyed by it."""
    h = hashlib.sha1()
    files = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp", ".h")))
    for path in files + [os.path.join(INCLUDE, "jacc.h")]:
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


def _compile(src, bid):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    flags = [*COMMON, f'-DJACC_BUILD_ID="{bid}"']
    cmd = ["hipcc", *flags, "-c", src, "-o", obj]
    if src.endswith(".hip"):
        cmd = ["hipcc", "-x", "hip", *flags, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=False, asan=False):
    """Compiles every source and links the library.  asan=True builds a
    second library, libjacc_asan.so, whose host code (the runtime) carries
    AddressSanitizer checks (device code is built as usual); it is for the
    CPU tests, loaded through JACC_LIB with the sanitizer runtime preloaded."""
    global COMMON, BUILD
    saved = COMMON, BUILD
    lib = LIB
    link_extra = []
    if asan:
        COMMON = COMMON + ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
        BUILD = BUILD + "_asan"
        lib = os.path.join(HERE, "libjacc_asan.so")
        link_extra = ["-fsanitize=address", "-shared-libasan"]
    try:
        os.makedirs(BUILD, exist_ok=True)
        srcs = sources()
        bid = build_id()
        with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
            objs = list(ex.map(lambda src: _compile(src, bid), srcs))
        tmp = lib + ".tmp"
        cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *link_extra, *objs, "-o", tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        os.replace(tmp, lib)
    finally:
        COMMON, BUILD = saved
    if verbose:
        print(lib)
    return lib


if __name__ == "__main__":
    build(verbose=True, asan="--asan" in sys.argv[1:])
    sys.exit(0)
