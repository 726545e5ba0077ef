"""Compile the HIP library libbfmht.so in-tree for gfx950.

Usage: python -m paper_2605_21828_amd.build   (or build() from Python).
Always recompiles; the product never builds at import time.

`python -m paper_2605_21828_amd.build --asan` builds libbfmht_asan.so instead:
the same library with its host code (plan validation, device layout, call
checks) instrumented by AddressSanitizer, device code unchanged.  Load it with
BFMHT_LIB pointing at it and the sanitizer runtime preloaded (ASAN_RUNTIME
below); tests/test_asan_host.py runs the host-side ABI tests that way.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbfmht.so")
LIB_ASAN = os.path.join(HERE, "libbfmht_asan.so")
ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
SOURCES = ["plan.cpp", "kernels.hip", "lsqr.hip", "noalloc.hip", "factor.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def asan_runtime():
    """Path of the AddressSanitizer runtime that a process loading libbfmht_asan.so preloads."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    r = subprocess.run([hipcc, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return r.stdout.strip()


def build(verbose=False, asan=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    extra = ASAN_FLAGS if asan else []
    out = LIB_ASAN if asan else LIB
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(CSRC, "_" + os.path.splitext(s)[0] + ("_asan" if asan else "") + ".o")
        cmd = [hipcc] + HIPCC_FLAGS + extra + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s%s" % (s, r.stdout, r.stderr))
        objs.append(obj)
    tmp = out + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + extra + ["-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s%s" % (r.stdout, r.stderr))
    os.replace(tmp, out)
    for o in objs:
        os.remove(o)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, asan="--asan" in sys.argv))
