"""Build the HIP library (libadc.so) for gfx950 in-tree.

Usage: python -m paper_2012_06714_amd.build  (or build() from Python).
Every source under csrc/ is compiled with hipcc; objects are cached by
content hash in _build/ and linked against rocBLAS and rocSOLVER.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libadc.so")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", f"-I{ROCM}/include"]


def _sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def _headers_hash():
    h = hashlib.sha256()
    for d in (CSRC, os.path.join(os.path.dirname(HERE), "include")):
        for f in sorted(os.listdir(d)):
            if f.endswith((".hpp", ".h")):
                h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def _compile(src, hh):
    data = open(src, "rb").read()
    key = hashlib.sha256(data + hh.encode() + " ".join(FLAGS).encode()).hexdigest()[:20]
    obj = os.path.join(BUILD, os.path.basename(src) + "." + key + ".o")
    if not os.path.exists(obj):
        cmd = [f"{ROCM}/bin/hipcc", *FLAGS, "-c", src, "-o", obj + ".tmp"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        os.replace(obj + ".tmp", obj)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(OUT_DIR, exist_ok=True)
    hh = _headers_hash()
    srcs = _sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, hh), srcs))
    tmp = LIB + ".tmp"
    cmd = [f"{ROCM}/bin/hipcc", "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs,
           f"-L{ROCM}/lib", "-lrocblas", "-lrocsolver", f"-Wl,-rpath,{ROCM}/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
