"""Compile the HIP library for gfx950 into ``paper_2602_23040_amd/libpackuvgs.so``.

Every translation unit under ``csrc/`` is compiled with hipcc (in parallel)
and linked into one shared library exporting the C ABI of
``include/packuv_gs.h``.  Flags:

* ``--offload-arch=gfx950``: MI355X only.
* ``-ffp-contract=off``: no implicit FMA contraction; the projection relies
  on a fixed FP64 evaluation order, the compositing kernels use explicit
  ``fmaf`` so forward and adjoint take identical decisions.
* ``-munsafe-fp-atomics``: hardware float atomics for gradient sums.
* ``-Xclang -target-feature -Xclang -packed-fp32-ops``: packed FP32 vector
  instructions are kept out of the generated code.
* ``-mllvm -structurizecfg-skip-uniform-regions=1`` (render.hip only):
  branches on wave-uniform values stay unstructured (see EXTRA_FLAGS).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libpackuvgs.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
SOURCES = ["api.hip", "scan.hip", "fetch.hip", "quant.hip", "loss.hip", "uvprune.hip", "project.hip", "binsort.hip", "render.hip", "optim.hip"]
# Per-file flags.  render.hip: branches on wave-uniform values (the adjoint's
# per-entry block and clamp dispatch) are left unstructured.  Structurized, they
# became flow blocks that kept each pixel's transmittance and colour-behind
# state in two register sets, with two copies per skipped block and entry.
EXTRA_FLAGS = {"render.hip": ["-mllvm", "-structurizecfg-skip-uniform-regions=1"]}


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *EXTRA_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, len(SOURCES))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
