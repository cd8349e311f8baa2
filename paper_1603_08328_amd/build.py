"""Builds liblexp.so in-tree: HIP kernels and the C ABI for gfx950 with hipcc,
the host-only pieces (random numbers, proposers, max-flow, thread pool) with
g++.  Every call compiles from scratch.

Device code: -O3, -ffp-contract=off (fused multiply-adds only where fmaf() is
written), packed FP32 instructions disabled.  Host code: -O3 -ffp-contract=off
so the double-precision proposer arithmetic is rounded as written.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "liblexp.so")
ARCH = os.environ.get("LEXP_OFFLOAD_ARCH", "gfx950")


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False, csrc: str = CSRC, out: str = LIB) -> str:
    """Compiles the sources in `csrc` into the shared library `out` (default:
    the package's sources and its in-tree library)."""
    hipcc = _hipcc()
    tmp = tempfile.mkdtemp(prefix="lexp_build_")
    try:
        host_obj = os.path.join(tmp, "lexp_host.o")
        _run(["g++", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
              "-I", INCLUDE, "-c", os.path.join(csrc, "lexp_host.cpp"), "-o", host_obj], verbose)
        objs = [host_obj]
        for src in ("lexp_kernels.hip", "lexp_cut.hip", "lexp_post.hip", "lexp_net.hip", "lexp_api.hip"):
            obj = os.path.join(tmp, src.replace(".hip", ".o"))
            _run([hipcc, "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
                  "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                  "-Wall", "-Wno-unused-result", "-I", INCLUDE, "-I", csrc,
                  "-c", os.path.join(csrc, src), "-o", obj], verbose)
            objs.append(obj)
        out_tmp = out + ".tmp"
        _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out_tmp] + objs + ["-lpthread"], verbose)
        os.replace(out_tmp, out)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return out


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
