"""Compile the HIP library ``libsnnc.so`` for gfx950 with hipcc (in-tree).

Every source is compiled to its own object in parallel (the translation units
share no device symbols: each launches its own kernels), then linked.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsnnc.so")
SOURCES = ["api.hip", "gen.hip", "scan.hip", "sort.hip", "prepare.hip", "spikes.hip", "views.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-fp32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def build(verbose: bool = False) -> str:
    """Compile every source into libsnnc.so (always recompiles)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    with tempfile.TemporaryDirectory(prefix="snnc_build_") as tmpdir:
        objs, procs = [], []
        for s in SOURCES:
            obj = os.path.join(tmpdir, os.path.splitext(s)[0] + ".o")
            cmd = [hipcc, *FLAGS, "-c", "-o", obj, os.path.join(CSRC, s)]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        failed = []
        for s, p in procs:
            out, _ = p.communicate()
            if p.returncode != 0:
                failed.append(s)
                sys.stderr.write(out)
            elif verbose and out.strip():
                sys.stderr.write(out)
        if failed:
            raise RuntimeError(f"hipcc failed on {', '.join(failed)}")
        tmp = LIB + ".tmp"
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libsnnc.so")
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
