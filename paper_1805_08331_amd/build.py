"""Build the pdsink HIP library in-tree for gfx950 with hipcc.

``python -m paper_1805_08331_amd.build`` (or ``build()``) compiles
``csrc/pdsink_api.hip`` (the C ABI and the plain kernels),
``csrc/pdsink_bounds.hip`` (the kernel variant with the error-control bounds)
and ``csrc/pdsink_log.hip`` (the log-domain path for flagged pairs), one
process per translation unit, and links ``paper_1805_08331_amd/libpdsink.so``.
It always recompiles.  ``--profile`` builds ``libpdsink_prof.so`` instead,
with the phase cycle counters of the resident-kernel path (PDSINK_PROFILE=1).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpdsink.so")
LIB_PROF = os.path.join(HERE, "libpdsink_prof.so")
SOURCES = ["pdsink_api.hip", "pdsink_bounds.hip", "pdsink_log.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions stay off (the compiler would otherwise form them)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))


def build(verbose: bool = False, profile: bool = False) -> str:
    out = LIB_PROF if profile else LIB
    defs = ["-DPDSINK_PROFILE=1"] if profile else []
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objs = [out + "." + os.path.splitext(s)[0] + ".o" for s in srcs]
    cmds = [[hipcc(), *HIPCC_FLAGS, *defs, "-c", "-o", o, os.path.join(CSRC, s)] for s, o in zip(srcs, objs)]
    try:
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            list(ex.map(lambda c: _run(c, verbose), cmds))
        tmp = out + ".tmp"
        _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
        os.replace(tmp, out)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return out


if __name__ == "__main__":
    print(build(verbose=True, profile="--profile" in sys.argv[1:]))
