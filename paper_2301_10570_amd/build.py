"""Compile the HIP sources into the in-tree shared library libmspfmm.so (gfx950).

    python paper_2301_10570_amd/build.py

Each source is compiled to an object file in a private build folder (in
parallel), then the objects are linked.  Packed FP32 instructions are disabled
for device code (-packed-fp32-ops).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmspfmm.so")
SOURCES = ["api.hip", "tree.hip", "fgt.hip", "p2p.hip", "partner.hip", "backward.hip", "batch.hip",
           "descent.hip", "noalloc.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def compile_flags() -> list[str]:
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I", os.path.join(HERE, "..", "include")]


def build(verbose: bool = False, jobs: int | None = None) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    jobs = jobs or min(len(srcs), max(1, min(os.cpu_count() or 1, 16)))
    tmpdir = tempfile.mkdtemp(prefix="mspfmm_build_")
    try:
        objs, running = [], []
        failed = []

        def reap(block: bool):
            for item in list(running):
                proc, src = item
                if block or proc.poll() is not None:
                    out, err = proc.communicate()
                    running.remove(item)
                    if proc.returncode != 0:
                        failed.append((src, out + err))

        for src in srcs:
            obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
            objs.append(obj)
            cmd = [hipcc()] + compile_flags() + ["-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            while len(running) >= jobs:
                reap(False)
                if len(running) >= jobs:
                    running[0][0].wait()
            running.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True), src))
        reap(True)
        if failed:
            for src, log in failed:
                sys.stderr.write(f"--- {src}\n{log}")
            raise RuntimeError("hipcc failed building libmspfmm.so")
        tmp = LIB + f".tmp{os.getpid()}"
        cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("linking libmspfmm.so failed")
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
