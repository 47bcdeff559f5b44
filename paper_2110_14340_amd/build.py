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


def build(verbose=False, sanitizer=None):
    """Compiles every source and links the library.  sanitizer = "address"
    or "undefined" builds a second library, libjacc_asan.so or
    libjacc_ubsan.so, whose host code (the runtime) carries that
    sanitizer's checks (device code is built as usual); it is for the CPU
    tests, loaded through JACC_LIB with the sanitizer's runtime preloaded."""
    global COMMON, BUILD
    saved = COMMON, BUILD
    lib = LIB
    link_extra = []
    if sanitizer:
        tag = {"address": "asan", "undefined": "ubsan"}[sanitizer]
        COMMON = COMMON + ["-Xarch_host", f"-fsanitize={sanitizer}", "-Xarch_host", "-fno-omit-frame-pointer"]
        if sanitizer == "undefined":
            COMMON = COMMON + ["-Xarch_host", "-fno-sanitize-recover=all"]
        BUILD = BUILD + "_" + tag
        lib = os.path.join(HERE, f"libjacc_{tag}.so")
        link_extra = [f"-fsanitize={sanitizer}", "-shared-libsan"]
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
    args = sys.argv[1:]
    build(verbose=True, sanitizer="address" if "--asan" in args else "undefined" if "--ubsan" in args else None)
    sys.exit(0)
