"""Build libsorlayout.so (HIP for gfx950) and the benchmark's calibration
library libslprobe.so in place.

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
           os.path.join(CSRC, "sl_sym.hip"), os.path.join(CSRC, "sl_api.hip"),
           os.path.join(CSRC, "sl_noalloc.hip")]
PROBE_LIB = os.path.join(PKG, "libslprobe.so")
PROBE_SOURCES = [os.path.join(CSRC, "sl_probe.hip")]
DEPS = SOURCES + [os.path.join(CSRC, "sl_internal.h"), os.path.join(CSRC, "sl_device.h"),
                  os.path.join(INCLUDE, "sorlayout.h")]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


BUILD_DIR = os.path.join(PKG, "_build")


def flags() -> list:
    return [
        "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
        # packed FP32 instructions stay off: ordinary float code only
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-I", INCLUDE, "-I", CSRC,
    ]


def command(out: str = LIB, sources=None) -> list:
    """One hipcc line that compiles and links the whole library."""
    return [hipcc()] + flags() + ["-shared", "-o", out] + (SOURCES if sources is None else sources)


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in DEPS)


def _run(cmd: list, verbose: bool) -> None:
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    lines = [ln for ln in proc.stdout.splitlines() if "packed-fp32-ops" not in ln]
    if proc.returncode != 0:
        raise RuntimeError("hipcc failed (%d):\n%s" % (proc.returncode, "\n".join(lines)))
    if verbose and lines:
        print("\n".join(lines), flush=True)


def _compile(lib: str, sources: list, verbose: bool) -> None:
    """Each source to an object (in parallel), then one link."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(BUILD_DIR, exist_ok=True)
    tag = "%d" % os.getpid()
    objs = [os.path.join(BUILD_DIR, os.path.basename(src) + "." + tag + ".o") for src in sources]
    jobs = [[hipcc()] + flags() + ["-c", "-o", obj, src] for src, obj in zip(sources, objs)]
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", "0")) or (os.cpu_count() or 1), 16))
    try:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            for f in [ex.submit(_run, cmd, verbose) for cmd in jobs]:
                f.result()
        tmp = lib + ".tmp" + tag
        # every symbol resolved at link time: a missing definition fails the build, not the first load
        _run([hipcc(), "--offload-arch=" + ARCH, "-fPIC", "-shared", "-Wl,--no-undefined", "-o", tmp] + objs, verbose)
        os.replace(tmp, lib)
    finally:
        for obj in objs:
            if os.path.exists(obj):
                os.remove(obj)


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile both libraries (always when force, else only when sources are newer)."""
    if force or stale():
        _compile(LIB, SOURCES, verbose)
    if force or not os.path.exists(PROBE_LIB) or \
            os.path.getmtime(PROBE_LIB) < max(os.path.getmtime(p) for p in PROBE_SOURCES):
        _compile(PROBE_LIB, PROBE_SOURCES, verbose)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
