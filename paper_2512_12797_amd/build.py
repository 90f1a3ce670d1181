"""Build the gfx950 shared library ``libfwi_mi355.so`` in-tree with hipcc.

Usage: ``python -m paper_2512_12797_amd.build`` (or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfwi_mi355.so")
ROOT = os.path.dirname(HERE)

SOURCES = ["fwi_kernels.hip", "fwi_host.cpp", "fwi_static.hip", "nn_kernels.hip", "daps_kernels.hip", "svgd_kernels.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# packed FP32 instructions are disabled for all device code: some of their forms have given
# wrong results now and then on this hardware; hipcc -O3 would otherwise emit them by itself
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
# the compiler's per-kernel resource report: a kernel whose private arrays or spills land
# in scratch memory serialises on it, so any scratch use fails the build
RESOURCE = ["-Rpass-analysis=kernel-resource-usage"]


def scratch_users(report: str) -> list:
    """(kernel, bytes per lane) of every kernel with scratch memory in a resource report."""
    out, name = [], None
    for line in report.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name is not None and int(m.group(1)) > 0:
            out.append((name, int(m.group(1))))
    return out


def build(verbose: bool = False) -> str:
    """Compile every source and link the library.  Always recompiles."""
    objs = []
    tmpdir = os.path.join(HERE, "_build")
    os.makedirs(tmpdir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(tmpdir, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC] + COMMON + DEVICE_FLAGS + RESOURCE + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        # hipcc's host pass warns that it does not know the packed-fp32 feature: harmless
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                        if "packed-fp32-ops" not in l and "kernel-resource-usage" not in l)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s" % (src, msg))
        spills = scratch_users(r.stderr)
        if spills:
            raise RuntimeError("%s: kernels using scratch memory: %s" % (src, spills))
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
