"""Builds the HIP library ``liblskum.so`` for gfx950 in-tree with hipcc."""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = [os.path.join(HERE, "csrc", f) for f in
           ("lskum_device.hip", "lskum_api.hip", "lskum_mlp.hip", "lskum_mlp_api.hip")]
HEADERS = [os.path.join(HERE, "csrc", f) for f in
           ("lskum_internal.h", "lskum_math.h", "lskum_math_coef.h", "lskum_mlp.h",
            "lskum_tiles.h")] + \
          [os.path.join(os.path.dirname(HERE), "include", "lskum.h")]
LIB = os.path.join(HERE, "liblskum.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed fp32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
# Per-source additions.  The solver kernels evaluate exp/erf polynomials
# inside their neighbour loops; machine-level loop-invariant code motion
# hoists every double coefficient of them into a vector register pair, which
# then costs a register copy before each Horner step and 50-60 registers per
# lane (the residual needs 221 and runs two wavefronts per SIMD).  Without it
# the coefficients stay scalar operands: 160 registers, three wavefronts, and
# the residual and sweep kernels 8-10% faster.
SOURCE_FLAGS = {"lskum_device.hip": ["-mllvm", "-disable-machine-licm"]}


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
    h.update(repr((HIPCC_FLAGS, SOURCE_FLAGS)).encode())
    for f in SOURCES + HEADERS:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False) -> str:
    """Compiles the library (always) and returns its path: one object per
    source (in parallel, each with its own additions), then one link."""
    tmp = LIB + ".tmp"
    objdir = tempfile.mkdtemp(prefix="lskum_build_")
    try:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(objdir, os.path.basename(src) + ".o")
            cmd = [hipcc(), *HIPCC_FLAGS, *SOURCE_FLAGS.get(os.path.basename(src), []),
                   f'-DLSKUM_BUILD_HASH="{source_hash()}"',
                   "-I", os.path.join(os.path.dirname(HERE), "include"), "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            objs.append(obj)
            procs.append((cmd, subprocess.Popen(cmd)))
        failed = [(cmd, pr.returncode) for cmd, pr in procs if pr.wait() != 0]
        if failed:  # every compile has ended before the objects' folder goes
            raise subprocess.CalledProcessError(failed[0][1], failed[0][0])
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    finally:
        shutil.rmtree(objdir, ignore_errors=True)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
