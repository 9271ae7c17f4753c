"""Build step of the HIP library: compiles csrc/ for gfx950 into
``paper_1908_04489_amd/libucp.so`` with hipcc.

Load this file by path (importlib), not as
``paper_1908_04489_amd.build``: importing the package binds the library,
which does not exist yet (or is stale) when a build is needed.

Flags: -O3, no FP contraction outside explicit fmaf (candidate positions and
grid nodes are plain binary64 sums and products), packed-FP32 instructions
disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libucp.so")
SOURCES = ["ucp_kernels.hip", "ucp_coding.hip", "ucp_w2.hip", "ucp_noalloc.hip", "ucp_probe.hip", "ucp_api.cpp", "ucp_server.cpp"]
ARCH = os.environ.get("UCP_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if p and os.path.exists(p):
            return p
    return "hipcc"


def flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    ]


def build(verbose: bool = False, out: str = LIB, extra=()) -> str:
    """Compile every source and link the shared library (always rebuilds);
    ``out`` and ``extra`` (more hipcc flags) serve alternative builds."""
    objs = []
    bdir = os.path.join(os.path.dirname(os.path.abspath(out)), "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(bdir, src + ".o")
        cmd = [hipcc()] + flags() + list(extra) + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".hip"):
            cmd.insert(1, "-xhip")
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
