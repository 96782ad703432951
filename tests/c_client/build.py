"""Compile the plain C client of the library (rlb_run.c) next to this file.

It is a host program built with gcc against include/rlb.h, the HIP runtime
and the in-tree librlb.so (found at run time through an rpath relative to
the executable), so the GPU
test can run it without Python in the loop.
"""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "rlb_run.c")
EXE = os.path.join(HERE, "rlb_run")
LIBDIR = os.path.join(ROOT, "paper_1211_3286_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build() -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROCM, "include"),
           SRC, "-o", EXE + ".tmp",
           "-L" + LIBDIR, "-l:librlb.so", "-Wl,-rpath,$ORIGIN/../../paper_1211_3286_amd",
           "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"C client build failed:\n{r.stdout}\n{r.stderr}")
    os.replace(EXE + ".tmp", EXE)
    return EXE


if __name__ == "__main__":
    print(build())
