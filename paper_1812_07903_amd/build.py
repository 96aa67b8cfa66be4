"""Build the slso HIP library (libslso.so) for gfx950 with hipcc.

Every ``csrc/*.hip`` file is compiled to an object in ``_build/`` and the
objects are linked into ``libslso.so`` next to this file. The CPU oracle's C
sources (if any) are not part of this library.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libslso.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in ordinary VGPRs: without it the accumulators of the
    # FP64 tile products are copied to and from AGPRs around every unrolled
    # step of their K loops
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wno-unused-command-line-argument",
    "-I", INCLUDE, "-I", CSRC,
]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True)
    out = "\n".join(ln for ln in p.stdout.splitlines()
                    if "packed-fp32-ops" not in ln)
    return p.returncode, out


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith(".hip"))


def build(verbose: bool = True, jobs: int | None = None) -> str:
    """Compile every HIP source and link libslso.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    objs = [os.path.join(BUILD, os.path.basename(s)[:-4] + ".o") for s in srcs]
    jobs = jobs or min(8, len(srcs))

    def one(pair):
        src, obj = pair
        return src, _run([HIPCC, *FLAGS, "-c", src, "-o", obj])

    failed = []
    with cf.ThreadPoolExecutor(jobs) as ex:
        for src, (rc, out) in ex.map(one, zip(srcs, objs)):
            if verbose and out.strip():
                print(f"[slso build] {os.path.basename(src)}:\n{out}")
            if rc != 0:
                failed.append(src)
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(failed))
    tmp = LIB + ".tmp"
    rc, out = _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}",
                    *objs, "-pthread", "-o", tmp])
    if rc != 0:
        raise RuntimeError("link failed:\n" + out)
    shutil.move(tmp, LIB)
    if verbose:
        print(f"[slso build] wrote {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
