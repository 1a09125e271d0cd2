"""Build the HIP C-ABI library ``libnedf.so`` in-tree for gfx950.

The sources (``csrc/`` and ``include/``) are first copied into
``_build/src/``, so that hipcc's host and device passes, which read a file
separately, see the same text even if the tree changes during the build.
Each translation unit is compiled into ``_build/`` (in parallel), then linked
into ``paper_2308_04669_amd/libnedf.so``.  Run as
``python -m paper_2308_04669_amd.build``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libnedf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SNAP = os.path.join(BUILD, "src")
SNAP_CSRC = os.path.join(SNAP, "csrc")
SNAP_INCLUDE = os.path.join(SNAP, "include")

DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{SNAP_INCLUDE}", f"-I{SNAP_CSRC}", "-Wall", "-Wno-unused-function",
          "-Wno-unused-result"]


def _snapshot():
    if os.path.isdir(SNAP):
        shutil.rmtree(SNAP)
    shutil.copytree(CSRC, SNAP_CSRC)
    shutil.copytree(INCLUDE, SNAP_INCLUDE)


def _sources():
    out = []
    for f in sorted(os.listdir(SNAP_CSRC)):
        if f.endswith(".hip") or f.endswith(".cpp"):
            out.append(os.path.join(SNAP_CSRC, f))
    return out


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if src.endswith(".hip"):
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-x", "hip", *COMMON, *DEVICE_FLAGS, "-c", src, "-o", obj]
    else:
        cmd = [HIPCC, *COMMON, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in ln]
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n" + "\n".join(msgs))
    if msgs:
        sys.stderr.write("\n".join(msgs) + "\n")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    _snapshot()
    srcs = _sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
