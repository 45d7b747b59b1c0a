"""Build libspaqr.so for gfx950 in-tree (hipcc, no GPU needed).

    python -m paper_2102_09878_amd.build [--jobs N] [--debug]

Objects go to ``paper_2102_09878_amd/_build/``; the library is written to
``paper_2102_09878_amd/libspaqr.so``.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libspaqr.so")
ARCH = os.environ.get("SPAQR_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result", f"-I{os.path.join(ROOT, 'include')}"]
# packed FP32 instructions stay disabled in every device build
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]

SOURCES = ["analyze.cpp", "graph_nd.cpp", "capi.cpp", "solve.cpp", "tune.cpp", "factor.hip", "kernels.hip", "qr.hip", "pqr.hip", "apply.hip", "cgls.hip", "adjoint.hip", "noalloc.hip"]


def _compile(src: str, debug: bool) -> str:
    obj = os.path.join(OUT, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    opt = ["-g"] if debug else []
    if src.endswith(".hip"):
        cmd = [HIPCC, "-x", "hip", *DEVICE, *COMMON, *opt, "-c", path, "-o", obj]
    else:
        cmd = [HIPCC, *COMMON, *opt, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if warn:
        sys.stderr.write(f"[{src}] {warn}\n")
    return obj


def build(jobs: int | None = None, debug: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, debug), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--debug", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.debug))
