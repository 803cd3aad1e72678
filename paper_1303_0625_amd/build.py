"""Build step of the gfx950 library (hipcc, in-tree).

Produces ``paper_1303_0625_amd/liblbm.so`` from ``csrc/``.  Every HIP source is
compiled for gfx950 only, with packed-FP32 instruction selection disabled.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = [os.path.join(HERE, "csrc", "lbm_capi.hip"), os.path.join(HERE, "csrc", "nn_capi.hip"),
           os.path.join(HERE, "csrc", "lbm3d_capi.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def source_hash(family: str = "lbm") -> str:
    """Short hash of one kernel family's sources (ties a measurement to that
    kernel version): "lbm" = the two-dimensional solver files, "lbm3d" = the
    D3Q19 files, "nn" = the network."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.startswith(family + "_") and f.endswith((".h", ".hip")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def build_library(verbose: bool = False) -> str:
    """Compile liblbm.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{out}")
    if verbose and out.strip():
        print(out)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
