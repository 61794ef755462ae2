"""Build libsorlayout.so (HIP for gfx950) in place.

usage: python -m paper_1711_01228_amd.build_lib [--force]
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsorlayout.so")
SOURCES = [os.path.join(CSRC, "sl_kernels.hip"), os.path.join(CSRC, "sl_apsp.hip"), os.path.join(CSRC, "sl_batch.hip"),
           os.path.join(CSRC, "sl_exact.hip"), os.path.join(CSRC, "sl_weighted.hip"), os.path.join(CSRC, "sl_diff.hip"),
           os.path.join(CSRC, "sl_sym.hip"), os.path.join(CSRC, "sl_probe.hip"), os.path.join(CSRC, "sl_api.hip")]
DEPS = SOURCES + [os.path.join(CSRC, "sl_internal.h"), os.path.join(CSRC, "sl_device.h"),
                  os.path.join(INCLUDE, "sorlayout.h")]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def command(out: str = LIB) -> list:
    return [
        hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
        # packed FP32 instructions stay off: ordinary float code only
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-I", INCLUDE, "-I", CSRC, "-o", out,
    ] + SOURCES


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in DEPS)


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile the library (always when force, else only when sources are newer)."""
    if not force and not stale():
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    lines = [ln for ln in proc.stdout.splitlines() if "packed-fp32-ops" not in ln]
    if proc.returncode != 0:
        raise RuntimeError("hipcc failed (%d):\n%s" % (proc.returncode, "\n".join(lines)))
    if verbose and lines:
        print("\n".join(lines), flush=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
