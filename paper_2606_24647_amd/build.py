"""Build libgq.so (and libgqgen.so, the device input generator) for gfx950.

    python -m paper_2606_24647_amd.build

Every .hip file under csrc/ except gen.hip is compiled with hipcc for gfx950
and linked into paper_2606_24647_amd/libgq.so; gen.hip alone becomes
libgqgen.so.  Object files go to _build/ at the repository root.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]

LIB = os.path.join(PKG, "libgq.so")
GENLIB = os.path.join(PKG, "libgqgen.so")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def _link(objs, out):
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)


def build(verbose: bool = True) -> None:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = dict(zip(srcs, ex.map(_compile, srcs)))
    gen = [o for s, o in objs.items() if os.path.basename(s) == "gen.hip"]
    main = [o for s, o in objs.items() if os.path.basename(s) != "gen.hip"]
    _link(main, LIB)
    if gen:
        _link(gen, GENLIB)
    if verbose:
        print(f"built {LIB}" + (f" and {GENLIB}" if gen else ""))


if __name__ == "__main__":
    build()
    sys.exit(0)
