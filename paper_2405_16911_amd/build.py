"""Builds libcyclo.so (the HIP library) in-tree for gfx950 with hipcc.

Usage: python -m paper_2405_16911_amd.build   (or call build_library()).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libcyclo.so")
SOURCES = ["cyclo_kernels.hip", "cyclo_runtime.hip", "cyclo_batch.hip", "cyclo_nn.hip", "cyclo_grid.hip", "cyclo_scf.hip", "cyclo_window.hip", "cyclo_cfe.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    errs = [ln for ln in res.stderr.splitlines() if "packed-fp32-ops" not in ln]
    return res.returncode, errs


def build_library(verbose: bool = False) -> str:
    """Compiles every HIP source (one hipcc per file, in parallel) and links
    paper_2405_16911_amd/libcyclo.so; returns its path."""
    inc = ["-I", os.path.join(ROOT, "include")]
    with tempfile.TemporaryDirectory(prefix="cyclo_build_") as tmpd:
        objs, cmds = [], []
        for src in SOURCES:
            obj = os.path.join(tmpd, src + ".o")
            objs.append(obj)
            cmds.append([hipcc()] + HIPCC_FLAGS + inc + ["-c", os.path.join(CSRC, src), "-o", obj])
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
            results = list(ex.map(_run, cmds))
        for (rc, errs), src in zip(results, SOURCES):
            if rc != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n" + "\n".join(errs))
            if verbose and errs:
                print("\n".join(errs), file=sys.stderr)
        tmp = LIB + ".tmp"
        link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(link), flush=True)
        rc, errs = _run(link)
        if rc != 0:
            raise RuntimeError("link failed:\n" + "\n".join(errs))
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
