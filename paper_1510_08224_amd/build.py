"""Build the HIP library ``liblbm.so`` for gfx950 in-tree.

    python -m paper_1510_08224_amd.build

Compiles ``csrc/*.hip`` with hipcc into ``paper_1510_08224_amd/liblbm.so``,
and ``csrc/host_check.cpp`` with a sanitized copy of the runtime's host code
into ``paper_1510_08224_amd/lbm_host_check``.  Every HIP source is built
with packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = ["lbm_kernels.hip", "lbm_api.hip"]
PROBE_LIB = os.path.join(HERE, "libbwprobe.so")
PROBE_SOURCES = ["bw_probe.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# -ffp-contract=off: every kernel rounds each operation as written, so the
# same step gives bitwise the same populations in every kernel that inlines
# it (single and fused steps, batches, graphs).
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


CLANG = os.environ.get("HOST_CXX", "/opt/rocm/lib/llvm/bin/clang++")
HOST_CHECK = os.path.join(HERE, "lbm_host_check")
# host code only: each sanitizer flag follows -Xarch_host on hipcc lines
_SAN = "-fsanitize=" + ",".join(("address", "undefined"))


def _run_all(cmds, verbose):
    procs = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
    for p, cmd in procs:
        if p.wait() != 0:
            raise RuntimeError("build step failed: " + " ".join(cmd))


def _host_check(verbose):
    """The runtime's host code under address and undefined-behaviour
    sanitizers, linked with the product's kernels into a check program
    (csrc/host_check.cpp) that drives every entry point."""
    bdir = os.path.join(HERE, "_build")
    api = os.path.join(bdir, "lbm_api_san.o")
    drv = os.path.join(bdir, "host_check.o")
    _run_all([
        [HIPCC, *[f for f in FLAGS if f != "-O3"], "-O1", "-g", "-Xarch_host", _SAN, "-Xarch_host",
         "-fno-sanitize-recover=all", "-c", os.path.join(CSRC, "lbm_api.hip"), "-o", api],
        [CLANG, "-O1", "-g", "-std=c++17", "-Wall", _SAN, "-fno-sanitize-recover=all",
         "-I", os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, "host_check.cpp"), "-o", drv],
    ], verbose)
    tmp = HOST_CHECK + ".tmp"
    _run_all([[CLANG, _SAN, "-o", tmp, drv, api, os.path.join(bdir, "lbm_kernels.o"),
               "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]], verbose)
    os.replace(tmp, HOST_CHECK)
    return HOST_CHECK


def _link(srcs, lib, verbose):
    objs = []
    procs = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    for src in srcs:
        obj = os.path.join(HERE, "_build", src.replace(".hip", ".o"))
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    for p, cmd in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed: " + " ".join(cmd))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    """Build liblbm.so (the product), libbwprobe.so (bandwidth ceilings)
    and lbm_host_check (the runtime's host code under sanitizers)."""
    _link(PROBE_SOURCES, PROBE_LIB, verbose)
    lib = _link(SOURCES, LIB, verbose)
    _host_check(verbose)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
