"""Build libcabs.so (HIP for gfx950) in-tree.

    python -m paper_1607_07395_amd.build [--jobs N] [--debug]

Every ``csrc/*.hip`` file is compiled to an object with hipcc for gfx950 and
the objects are linked into ``paper_1607_07395_amd/libcabs.so``.  Packed FP32
instructions are disabled for all device code.
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
SRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libcabs.so")
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags(debug: bool) -> list[str]:
    flags = [
        f"--offload-arch={ARCH}",
        "-std=c++17",
        "-fPIC",
        "-O1" if debug else "-O3",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"),
        "-Wno-unused-result",
    ]
    if debug:
        flags += ["-g"]
    return flags


def _compile(src: str, obj: str, debug: bool) -> tuple[str, int, str]:
    cmd = [hipcc(), "-c", src, "-o", obj] + common_flags(debug)
    p = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the GPU-only feature flag; drop that warning
    err = "\n".join(l for l in p.stderr.splitlines() if "packed-fp32-ops" not in l)
    return src, p.returncode, err


def build(jobs: int = 8, debug: bool = False, verbose: bool = True) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    sources = sorted(f for f in os.listdir(SRC) if f.endswith(".hip"))
    objs = []
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        futs = []
        for f in sources:
            obj = os.path.join(OUT_DIR, f[:-4] + ".o")
            objs.append(obj)
            futs.append(ex.submit(_compile, os.path.join(SRC, f), obj, debug))
        failed = False
        for fu in futs:
            src, rc, err = fu.result()
            if err.strip() and (verbose or rc):
                print(f"[{os.path.basename(src)}]\n{err}", file=sys.stderr)
            failed |= rc != 0
    if failed:
        raise RuntimeError("HIP compilation failed")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-o", tmp] + objs + [f"--offload-arch={ARCH}", "-fPIC", "-lpthread"]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--debug", action="store_true")
    a = ap.parse_args()
    build(a.jobs, a.debug)
