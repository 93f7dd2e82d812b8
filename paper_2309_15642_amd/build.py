"""Build libgpeps.so (HIP kernels + C ABI) in-tree for gfx950 with hipcc.

    python -m paper_2309_15642_amd.build

The library lands next to this file; the Python binding loads it from there.
Every HIP source is compiled with packed-FP32 instruction selection disabled.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgpeps.so")
SOURCES = ["gpeps_kernels.hip", "gpeps_bigbond.hip", "gpeps_adjoint.hip", "gpeps_bp.hip", "gpeps_host.cpp"]
PEAKS_SOURCE = "gpeps_peaks.hip"  # FP64 FMA / MFMA and copy probes for the benchmark (libgpeps_peaks.so)
PEAKS_LIB = os.path.join(HERE, "libgpeps_peaks.so")
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libgpeps")


def compile_flags() -> list:
    return [
        f"--offload-arch={ARCH}",
        "-O3",
        "-std=c++17",
        "-fPIC",
        "-Wall",
        "-Wno-unused-parameter",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        f"-I{os.path.join(ROOT, 'include')}",
        f"-I{CSRC}",
    ]


def build(verbose: bool = False) -> str:
    """Compile every source and link libgpeps.so; returns the library path."""
    cc = hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [cc, *compile_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd.insert(1, "-xhip")
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        noise = [ln for ln in (res.stderr or "").splitlines() if "packed-fp32-ops" not in ln]
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n" + "\n".join(noise))
        if verbose and noise:
            print("\n".join(noise), file=sys.stderr)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stderr)
    os.replace(tmp, LIB)
    # peak-rate probes used by the benchmark, a library of their own
    obj = os.path.join(objdir, "gpeps_peaks.o")
    res = subprocess.run([cc, *compile_flags(), "-c", os.path.join(CSRC, PEAKS_SOURCE), "-o", obj],
                         capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {PEAKS_SOURCE}:\n" + res.stderr)
    res = subprocess.run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", PEAKS_LIB + ".tmp", obj],
                         capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stderr)
    os.replace(PEAKS_LIB + ".tmp", PEAKS_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
