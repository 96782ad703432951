"""Build ``librlb.so`` (the HIP kernels and the C ABI of include/rlb.h) for gfx950.

Every source is compiled with hipcc for gfx950 only, with packed FP32 ops
disabled, into position-independent objects linked into one shared library
that sits next to this file.

The build refuses any kernel that uses scratch (private) memory, i.e. that
spills registers: the compiler's kernel resource report is read for every
kernel of every source, and a ScratchSize above zero fails the build with the
kernels named. Spilled builds are the class that once returned wrong results
from a graph-launched persistent kernel (FP64, 1024 threads, general equation
of state), and no kernel here needs scratch otherwise.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "librlb.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["kernels.hip", "kernels2d.hip", "adjoint.hip", "noalloc.hip", "api.cpp"]
HEADERS = ["cell.hpp", "cell2d.hpp", "adjoint_cell.hpp", "device_util.hpp", "internal.hpp",
           "adjoint.hpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(HERE, "..", "include")]


def scratch_users(report: str) -> dict:
    """Kernels with a nonzero ScratchSize in hipcc's
    -Rpass-analysis=kernel-resource-usage output: {mangled name: bytes per lane}."""
    out, name = {}, None
    for line in report.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name and int(m.group(1)) > 0:
            out[name] = int(m.group(1))
    return out


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj,
           "-Rpass-analysis=kernel-resource-usage"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    users = scratch_users(r.stderr)
    if users:
        names = "\n".join(f"  {k}: {v} B/lane" for k, v in sorted(users.items()))
        raise RuntimeError(f"{src}: kernels that use scratch memory (register spills) are "
                           f"refused:\n{names}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", OUT + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
