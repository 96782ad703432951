"""The plain C client of the ABI (tests/c_client/rlb_run.c) builds and links
against librlb.so and the HIP runtime, rejects a bad command line, and, with
no GPU, stops at its first device call (hipMalloc, after rlb_workspace_size
has sized the workspace) with a named error."""

import os
import subprocess
import tempfile

import numpy as np
import pytest

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_client", "rlb_run")


def _need_exe():
    if not os.path.exists(EXE):
        pytest.fail("tests/c_client/rlb_run is not built (run __graft_entry__.build())")


def test_usage_error():
    _need_exe()
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "usage" in r.stderr


def test_stops_at_the_first_device_call_without_a_gpu():
    _need_exe()
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present: the GPU test runs the client")
    except ImportError:
        pass
    d = tempfile.mkdtemp()
    nc = 4 * 3 * 2
    np.concatenate([np.ones(nc), np.ones(nc), np.zeros(3 * nc)]).tofile(os.path.join(d, "in.bin"))
    r = subprocess.run([EXE, "4", "3", "2", "0", "0", "0", "0.8", "0.8", "0.6", "0.7", "0", "5",
                        os.path.join(d, "in.bin"), os.path.join(d, "out.bin")],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "hipMalloc failed" in r.stderr, r.stderr
