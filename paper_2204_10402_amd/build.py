"""Build libvc.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2204_10402_amd.build

hipcc cross-compiles for gfx950 without a GPU present. The library is written next to this
file as ``libvc.so``; the Python binding loads it from there.
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
LIB = os.path.join(PKG, "libvc.so")
SOURCES = ["vc_device.hip", "vc_bitset.hip", "vc_host.cpp", "vc_server.cpp", "vc_noalloc.hip"]
ARCH = os.environ.get("VC_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libvc.so)")


FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-pthread",
    # no packed-FP32 instructions anywhere (the library has no float arithmetic anyway)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def compile_command(src: str, obj: str) -> list[str]:
    return [hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]


def link_command(objs: list[str], out: str) -> list[str]:
    return [hipcc(), *FLAGS, "-shared", *objs, "-o", out]


def build(verbose: bool = False) -> str:
    """Compile every source to an object file (in parallel, one process per source), then
    link libvc.so. Objects go to a temporary directory; only the library stays in-tree."""
    from concurrent.futures import ThreadPoolExecutor
    tmp = LIB + ".tmp"
    with tempfile.TemporaryDirectory(prefix="vc_build_") as work:
        objs = [os.path.join(work, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [compile_command(s, o) for s, o in zip(SOURCES, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with ThreadPoolExecutor(len(cmds)) as ex:
            for f in [ex.submit(subprocess.check_call, c, cwd=ROOT) for c in cmds]:
                f.result()
        cmd = link_command(objs, tmp)
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd, cwd=ROOT)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
