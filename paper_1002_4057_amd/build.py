"""Builds the HIP library ``libspdinv.so`` in place (gfx950 only).

Usage: ``python -m paper_1002_4057_amd.build``.  Every call recompiles.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libspdinv.so")
SOURCES = ["device.hip", "batched.hip", "mixed.hip", "dense.hip", "api.cpp", "plan.cpp"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    cc = hipcc()
    flags = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    tmpdir = tempfile.mkdtemp(prefix="spdinv_build_")
    try:
        objs = []
        for src in SOURCES:
            obj = os.path.join(tmpdir, src + ".o")
            cmd = [cc] + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"compiling {src} failed:\n{r.stderr}")
            objs.append(obj)
        tmp_lib = os.path.join(tmpdir, "libspdinv.so")
        cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}"] + objs + ["-o", tmp_lib]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"linking failed:\n{r.stderr}")
        os.replace(tmp_lib, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
