"""Compile the HIP sources under csrc/ into the in-tree shared library libgrf.so (gfx950)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
OBJ = PKG / "_build"
LIB = PKG / "libgrf.so"
PROBE_LIB = PKG / "libgrf_probe.so"
SOURCES = ["api.cpp", "modes.cpp", "tables.hip", "direct.hip", "sep.hip", "adjoint.hip", "batch.hip", "krige.hip", "noalloc.hip", "points.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", str(ROOT / "include"), "-I", str(CSRC)]


# Per-source flags: the binned point sum keeps its FP32 matrix-product results in ordinary
# VGPRs (the vector units read every element; accumulation registers would add a copy each).
EXTRA = {"points.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _compile(src: str) -> Path:
    out = OBJ / (src.replace(".", "_") + ".o")
    lang = ["-x", "hip"] if src.endswith((".hip", ".cpp")) else []
    cmd = [HIPCC, *FLAGS, *EXTRA.get(src, []), *lang, "-c", str(CSRC / src), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed for {src}")
    return out


def build(verbose: bool = False) -> Path:
    """Compile every source for gfx950 and link libgrf.so (always rebuilds)."""
    OBJ.mkdir(exist_ok=True)
    jobs = min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB.with_suffix(".so.tmp%d" % os.getpid())
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", str(tmp), *map(str, objs)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libgrf.so failed")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    # issue-rate probes of the benchmark (a library of their own, not part of the C ABI)
    pobj = _compile("probe.hip")
    tmp = PROBE_LIB.with_suffix(".so.tmp%d" % os.getpid())
    r = subprocess.run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", str(tmp), str(pobj)],
                       capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libgrf_probe.so failed")
    os.replace(tmp, PROBE_LIB)
    if verbose:
        print(f"built {PROBE_LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
