"""Builds the HIP library ``liblskum.so`` for gfx950 in-tree with hipcc."""
from __future__ import annotations

import hashlib
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = [os.path.join(HERE, "csrc", f) for f in
           ("lskum_device.hip", "lskum_api.hip", "lskum_mlp.hip", "lskum_mlp_api.hip")]
HEADERS = [os.path.join(HERE, "csrc", "lskum_internal.h"), os.path.join(HERE, "csrc", "lskum_mlp.h"),
           os.path.join(os.path.dirname(HERE), "include", "lskum.h")]
LIB = os.path.join(HERE, "liblskum.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed fp32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    return "hipcc"


def source_hash() -> str:
    """First 16 hex digits of the SHA-256 of the library's sources and headers;
    compiled into the library (lskum_build_hash) so that a stale binary is
    recognised by content, whatever the file times."""
    h = hashlib.sha256()
    for f in SOURCES + HEADERS:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False) -> str:
    """Compiles the library (always) and returns its path."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, f'-DLSKUM_BUILD_HASH="{source_hash()}"',
           "-I", os.path.join(os.path.dirname(HERE), "include"), *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
