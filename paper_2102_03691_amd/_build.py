"""Compile libmodalhc.so (HIP, gfx950) in-tree with hipcc.

Each source is compiled to an object on its own (in parallel), then the
objects are linked into the shared library; every call compiles everything.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmodalhc.so")
OBJ_DIR = os.path.join(ROOT, "_build")

SOURCES = ["mhc_api.cpp", "mhc_shc.cpp", "mhc_virial.cpp", "k_prep.hip", "k_contract.hip", "k_accum.hip", "k_shc.hip",
           "k_tersoff.hip"]

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # keep the compiler from emitting packed-FP32 VALU instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]

NOISE = "is not a recognized feature for this target"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if NOISE not in l)
    return r.returncode, err


def build(verbose: bool = False) -> str:
    """Compile every source into LIB; returns its path. Raises on failure."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    srcs = list(SOURCES)
    objs = [os.path.join(OBJ_DIR, os.path.splitext(s)[0] + ".o") for s in srcs]
    cmds = [[hipcc(), *FLAGS, "-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(srcs, objs)]
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1)), 16))
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_run, cmds))
    for (rc, err), s in zip(results, srcs):
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {s} ({rc}):\n{err}")
        if verbose and err.strip():
            print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    rc, err = _run(link)
    if rc != 0:
        raise RuntimeError(f"hipcc link failed ({rc}):\n{err}")
    os.replace(tmp, LIB)
    return LIB


# Host sanitizer build of the test drivers: the host translation units of the C
# ABI compiled with AddressSanitizer and UndefinedBehaviorSanitizer (host code
# only; the device code and the kernel objects are the normal build's), linked
# with the normal build's kernel objects into a separate library that two C99
# drivers (tests/c) load.  The drivers link the sanitizer runtimes themselves,
# so no preloading is needed.
HOST_TUS = ["mhc_api.cpp", "mhc_shc.cpp", "mhc_virial.cpp"]
ASAN_DIR = os.path.join(ROOT, "tests", "c", "build")
SAN_HOST = ["-g", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-fsanitize=address",
            "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined"]
DRIVERS = ["abi_run.c", "abi_errors.c"]


def clang() -> str:
    for cand in ("/opt/rocm/llvm/bin/clang", "clang"):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    return "clang"


def build_sanitized(verbose: bool = False) -> str:
    """Build tests/c/build/libmodalhc_asan.so and the sanitized C drivers; needs build() first."""
    os.makedirs(ASAN_DIR, exist_ok=True)
    dev_objs = [os.path.join(OBJ_DIR, os.path.splitext(s)[0] + ".o") for s in SOURCES if s not in HOST_TUS]
    missing = [o for o in dev_objs if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"kernel objects missing ({missing[0]}): run build() first")
    host_objs = [os.path.join(ASAN_DIR, os.path.splitext(s)[0] + ".o") for s in HOST_TUS]
    cmds = [[hipcc(), *FLAGS, *SAN_HOST, "-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(HOST_TUS, host_objs)]
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        results = list(ex.map(_run, cmds))
    for (rc, err), s in zip(results, HOST_TUS):
        if rc != 0:
            raise RuntimeError(f"sanitized hipcc failed on {s} ({rc}):\n{err}")
    lib = os.path.join(ASAN_DIR, "libmodalhc_asan.so")
    rc, err = _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *host_objs, *dev_objs, "-o", lib])
    if rc != 0:
        raise RuntimeError(f"sanitized link failed ({rc}):\n{err}")
    for d in DRIVERS:
        exe = os.path.join(ASAN_DIR, os.path.splitext(d)[0] + "_asan")
        cmd = [clang(), "-std=c99", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"),
               os.path.join(ROOT, "tests", "c", d), lib, "-Wl,-rpath," + ASAN_DIR, "-o", exe]
        if verbose:
            print(" ".join(cmd), flush=True)
        rc, err = _run(cmd)
        if rc != 0:
            raise RuntimeError(f"driver build failed ({d}, {rc}):\n{err}")
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_sanitized(verbose=True))
