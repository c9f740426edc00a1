"""Compile the HIP library libclbm.so for gfx950 (in-tree).

The library carries a hash of the sources it was built from (returned by
clbm_version()); the binding compares it with the sources in the tree and
refuses a stale library.
"""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libclbm.so")
SOURCES = [os.path.join(HERE, "csrc", f)
           for f in ("clbm_api.hip", "clbm_kernels.hip", "clbm_rows.hip", "clbm_fused.hip", "clbm_inplace.hip",
                     "clbm_batch.hip")]

# Packed FP32 instructions are disabled for every device compilation.
HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-command-line-argument"]


def source_hash() -> str:
    """Hash of every source the library is built from (kernels, runtime,
    the public header) and of the compiler flags."""
    h = hashlib.sha256()
    files = sorted(os.path.join(HERE, "csrc", f) for f in os.listdir(os.path.join(HERE, "csrc"))
                   if f.endswith((".hip", ".hpp", ".h")))
    files.append(os.path.join(ROOT, "include", "clbm.h"))
    for path in files:
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(HIPCC_FLAGS).encode())
    return h.hexdigest()[:16]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False) -> str:
    """Compile each source to an object (in parallel), then link the library."""
    tag = ".tmp%d" % os.getpid()
    objs = [os.path.join(HERE, "csrc", os.path.basename(src) + tag + ".o") for src in SOURCES]
    defs = ['-DCLBM_SOURCE_HASH="%s"' % source_hash()]
    cmds = [[hipcc()] + HIPCC_FLAGS + defs + ["-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj]
            for src, obj in zip(SOURCES, objs)]
    try:
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            for cmd in cmds:
                if verbose:
                    print(" ".join(cmd), flush=True)
            for r in ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds):
                if r.returncode != 0:
                    sys.stderr.write(r.stdout + r.stderr)
                    raise subprocess.CalledProcessError(r.returncode, r.args)
        tmp = LIB + tag
        link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
        os.replace(tmp, LIB)
    finally:
        for obj in objs:
            if os.path.exists(obj):
                os.remove(obj)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
