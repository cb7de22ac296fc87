"""Builds the in-tree shared library libuot.so for gfx950 with hipcc.

    python -m paper_1909_00149_amd.build        (from the repository root)

Every HIP source is compiled with packed-FP32 instruction generation turned
off (-Xclang -target-feature -Xclang -packed-fp32-ops); hipcc's host pass
warns that it does not know that feature, which is harmless.

Multiply-adds are fused only where one source expression holds both
(-ffp-contract=on).  hipcc's default lets the back end fuse across
statements, and it does so differently in differently shaped code (the
scalar kernel, and the full and partial quads of the vectorised kernel), so
kernels written with the same per-pixel formulas would round differently;
with expression-level fusion every tile shape computes every pixel
identically.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libuot.so")

ARCH = os.environ.get("UOT_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]

# (source, object name, extra defines); the fused-iteration kernels are
# instantiated once per mode from one source, so the three sets compile in
# parallel
SOURCES = [("uot_iter_mode.hip", "uot_iter_mode0", ["-DUOT_MODE=0"]),
           ("uot_iter_mode.hip", "uot_iter_mode1", ["-DUOT_MODE=1"]),
           ("uot_iter_mode.hip", "uot_iter_mode2", ["-DUOT_MODE=2"]),
           ("uot_kernels.hip", "uot_kernels", []), ("uot_poisson.hip", "uot_poisson", []),
           ("uot_dr.hip", "uot_dr", []),
           ("uot_host.cpp", "uot_host", []), ("uot_admm_kernels.hip", "uot_admm_kernels", []),
           ("uot_admm_host.cpp", "uot_admm_host", []), ("uotnet_kernels.hip", "uotnet_kernels", []),
           ("uotnet_host.cpp", "uotnet_host", [])]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def _compile(entry):
    src, name, defs = entry
    out = os.path.join(OBJ, name + ".o")
    lang = ["-x", "hip"] if src.endswith((".hip", ".cpp")) else []
    cmd = [hipcc(), *lang, *FLAGS, *defs, "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return out


def build(verbose=False):
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from paper_1909_00149_amd._lib import DIGEST_PATH, sources_digest
    digest = sources_digest()  # of the sources as they are when the compile starts
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(6, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    with open(DIGEST_PATH + ".tmp", "w") as f:
        f.write(digest + "\n")
    os.replace(DIGEST_PATH + ".tmp", DIGEST_PATH)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
