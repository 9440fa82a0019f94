"""Builds the gfx950 HIP library ``liblbmadj.so`` in place with hipcc.

Flags: ``-O3`` with IEEE float division/sqrt (no fast-math), ``-fPIC -shared``,
``-Xclang -target-feature -Xclang -packed-fp32-ops`` (packed FP32 VALU
instructions are turned off for all device code) and ``-ffp-contract=on``:
a multiply is fused into an add only inside one source expression, so the
fusion pattern is a property of the source, not of how a node function was
inlined.  The single-context and batched kernels share the node functions,
and with this flag they round identically (batched results are bitwise the
single-context ones).  The library links the profiler's marker library
(rocprofiler-sdk-roctx) for its named ranges.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbmadj.so")
SOURCES = [os.path.join(CSRC, "lbm_adj.hip")]
DEPS = SOURCES + [os.path.join(CSRC, f) for f in ("kernels.hpp", "lattice.hpp")] + [
    os.path.join(ROOT, "include", "lbm_adj.h")]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")
# profiler marker library (named ranges around forward, recompute and adjoint segments)
ROCM_LIB = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")


def hipcc() -> str:
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    return "hipcc"


def command(out: str = LIB, extra=()) -> list:
    return [hipcc(), "--offload-arch=%s" % ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=on",
            "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include"), *extra,
            "-o", out, *SOURCES, "-L", ROCM_LIB, "-Wl,-rpath," + ROCM_LIB, "-lrocprofiler-sdk-roctx"]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS)


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile the library (always when force, else only if missing or stale)."""
    if not force and not stale():
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    proc = subprocess.run(command(tmp), capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + proc.stdout + proc.stderr)
    if verbose:
        print(proc.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
