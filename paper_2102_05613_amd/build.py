"""Build the HIP libraries for gfx950 (in-tree, next to this file): libmc3.so, the
Monte Carlo path, and libmc3ceil.so, the matrix-core ceiling measurement."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmc3.so")
SOURCES = [os.path.join(CSRC, "mc3.hip")]
HEADERS = ([os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith(".hpp")]
           + [os.path.join(ROOT, "include", "mc3.h")])
LIB_CEIL = os.path.join(HERE, "libmc3ceil.so")
SOURCES_CEIL = [os.path.join(CSRC, "ceiling.hip")]
HEADERS_CEIL = [os.path.join(ROOT, "include", "mc3_ceiling.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # every FP64 operation of the selection rule is separately rounded
    "-ffp-contract=off",
    # no packed FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _compile(lib: str, sources, headers, force: bool, verbose: bool) -> str:
    if not force and os.path.exists(lib):
        newest = max(os.path.getmtime(p) for p in sources + headers)
        if os.path.getmtime(lib) >= newest:
            return lib
    tmp = lib + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp, *sources]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building " + os.path.basename(lib))
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(tmp, lib)
    return lib


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile libmc3.so and libmc3ceil.so with hipcc.  Always recompiles when force is
    true.  Returns the path of libmc3.so."""
    _compile(LIB_CEIL, SOURCES_CEIL, HEADERS_CEIL, force, verbose)
    return _compile(LIB, SOURCES, HEADERS, force, verbose)


if __name__ == "__main__":
    print(build(force=True, verbose=True))
