"""Compile the HIP library libcyrus.so for gfx950, in-tree.

Every source under csrc/ is compiled with hipcc (device code for gfx950 only)
and linked into paper_2506_00167_amd/libcyrus.so, which the Python binding
loads. Usage: python -m paper_2506_00167_amd.build [-v]
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcyrus.so")
ARCH = "gfx950"

SOURCES = ["cyrus_api.cpp", "cyrus_batch.cpp", "cyrus_engine.cpp", "cyrus_critic.cpp", "kernels_level.hip",
           "kernels_subtree.hip", "kernels_critic.hip"]

FLAGS = [
    "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off (they have given silently wrong
    # results on these parts); ordinary float code is scalar FMA instead
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
]


def source_hash() -> str:
    """SHA-256 (first 16 hex digits) of every file the library is compiled
    from: csrc/* and include/cyrus.h, in name order. It is compiled into the
    library, and the binding refuses a library whose hash differs from that of
    the sources beside it (a stale build)."""
    h = hashlib.sha256()
    files = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                   if f.endswith((".cpp", ".hip", ".h")))
    files.append(os.path.join(ROOT, "include", "cyrus.h"))
    for path in files:
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, verbose: bool, src_hash: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [_hipcc(), *FLAGS, f'-DCYRUS_SOURCE_HASH="{src_hash}"', "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    if verbose:
        noise = "is not a recognized feature for this target"
        msg = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
        if msg.strip():
            print(msg, file=sys.stderr)
    return obj


def build(verbose: bool = False) -> str:
    """Compile all sources and link libcyrus.so. Returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    src_hash = source_hash()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, src_hash), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
