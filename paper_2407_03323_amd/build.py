"""Build the HIP library libmotjvie.so for gfx950 (in-tree, next to this file)."""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmotjvie.so")
SOURCES = ["mj_fft.hip", "mj_gen.hip", "mj_march.hip", "mj_api.hip"]
ARCH = "gfx950"

HIPCC_FLAGS = [
    "-O3", "-std=c++20", "-fPIC",
    "--offload-arch=" + ARCH,
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


DIGEST = os.path.join(BUILD, "libmotjvie.sha1")


def source_digest() -> str:
    """SHA-1 of every source and header the library is built from, and of the compiler flags."""
    h = hashlib.sha1(" ".join(HIPCC_FLAGS).encode())
    files = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith((".hip", ".h"))]
    files += [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def built_digest():
    """Digest recorded by the last build (None if there is none)."""
    try:
        with open(DIGEST) as fh:
            return fh.read().strip()
    except OSError:
        return None


def is_current() -> bool:
    """The built library was compiled from the sources as they are now."""
    return os.path.exists(LIB) and built_digest() == source_digest()


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile every source for gfx950 and link the shared library; always recompiles."""
    os.makedirs(BUILD, exist_ok=True)
    digest = source_digest()
    objs = []
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    for src in SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        cmd = [hipcc()] + HIPCC_FLAGS + inc + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + ["-shared", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    with open(DIGEST + ".tmp", "w") as fh:
        fh.write(digest + "\n")
    os.replace(DIGEST + ".tmp", DIGEST)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
