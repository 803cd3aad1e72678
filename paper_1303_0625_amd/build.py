"""Build step of the gfx950 library (hipcc, in-tree).

Produces ``paper_1303_0625_amd/liblbm.so`` from ``csrc/``.  Every HIP source is
compiled for gfx950 only, with packed-FP32 instruction selection disabled; the
translation units compile in parallel and are linked into one shared library.
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
OBJDIR = os.path.join(HERE, "_build")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
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


def _clean(text: str) -> str:
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)


def build_library(verbose: bool = False) -> str:
    """Compile liblbm.so (always recompiles every translation unit)."""
    os.makedirs(OBJDIR, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, os.path.basename(src).replace(".hip", ".o"))
        cmd = [HIPCC, *FLAGS, "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                            text=True)))
        objs.append(obj)
    failed = []
    for cmd, p in procs:
        out, _ = p.communicate()
        out = _clean(out)
        if p.returncode != 0:
            failed.append(f"{' '.join(cmd)}\n{out}")
        elif verbose and out.strip():
            print(out)
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n".join(failed))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc link failed ({r.returncode}):\n{_clean(r.stdout + r.stderr)}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
