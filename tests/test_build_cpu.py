"""The build's refusal of kernels that use scratch memory (register spills).

paper_1211_3286_amd/build.py reads hipcc's kernel resource report for every
kernel and fails on a ScratchSize above zero. Checked here on a kernel made
to need scratch (a per-thread array indexed at run time) and on one that does
not, compiled for gfx950 with the library's own flags.
"""

import os
import shutil
import subprocess
import tempfile

import pytest

from paper_1211_3286_amd import build

SRC = r"""
#include <hip/hip_runtime.h>
__global__ __launch_bounds__(256) void k_private(const int* idx, float* out) {
  float a[64];
  for (int i = 0; i < 64; ++i) a[i] = out[threadIdx.x + i];
  out[threadIdx.x] = a[idx[threadIdx.x] & 63];
}
__global__ __launch_bounds__(256) void k_plain(const float* in, float* out) {
  out[threadIdx.x] = 2.0f * in[threadIdx.x];
}
"""


@pytest.mark.skipif(not os.path.exists(build.HIPCC), reason="hipcc not installed")
def test_scratch_users_are_found():
    d = tempfile.mkdtemp()
    try:
        src = os.path.join(d, "t.hip")
        with open(src, "w") as fh:
            fh.write(SRC)
        cmd = [build.HIPCC, *build.FLAGS, "-x", "hip", "-c", src, "-o", os.path.join(d, "t.o"),
               "-Rpass-analysis=kernel-resource-usage"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        users = build.scratch_users(r.stderr)
        assert any("k_private" in k for k in users), users
        assert not any("k_plain" in k for k in users), users
    finally:
        shutil.rmtree(d)


def test_scratch_report_parsing():
    rep = "\n".join([
        "a.hip:1:1: remark: Function Name: _Z3fooPf [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:1:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark: Function Name: _Z3barPf [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark:     ScratchSize [bytes/lane]: 332 [-Rpass-analysis=kernel-resource-usage]",
    ])
    assert build.scratch_users(rep) == {"_Z3barPf": 332}
