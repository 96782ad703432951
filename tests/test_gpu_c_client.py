"""The C ABI end to end from a plain C host program (tests/c_client/rlb_run.c):
it sizes and allocates the workspace, creates its stream, initialises from
host fields, steps and reads the fields back, with no Python in the loop.
Its output must equal the Python binding's run of the same lattice bit for
bit (the same library, the same default kernel) and match the FP64 oracle
within the step tests' tolerances (FP64 1e-12, FP32 1e-5)."""

import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_helpers import relmax, say

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_client", "rlb_run")
FP64, FP32 = 0, 1
TOL = {FP64: 1e-12, FP32: 1e-5}


def _run_client(prob, prec, T, d):
    p = prob.params
    nc = p.ncells
    np.concatenate([prob.n.ravel(), prob.eps.ravel(), prob.u.reshape(3, -1).ravel()]).astype(
        np.float64).tofile(os.path.join(d, "in.bin"))
    args = [EXE, str(p.nx), str(p.ny), str(p.nz), *[str(b) for b in p.bc],
            repr(p.tau_f), repr(p.tau_v), repr(p.tau_e), repr(p.tau_eps), str(prec), str(T),
            os.path.join(d, "in.bin"), os.path.join(d, "out.bin")]
    say("c client", " ".join(args[1:13]))
    r = subprocess.run(args, capture_output=True, text=True, timeout=120)
    say(r.stdout.strip(), r.stderr.strip())
    assert r.returncode == 0, r.stderr
    raw = np.fromfile(os.path.join(d, "out.bin"), dtype=np.float64)
    assert raw.size == 7 * nc + 5 + 1
    return {"n": raw[:nc], "eps": raw[nc:2 * nc], "P": raw[2 * nc:3 * nc],
            "gamma": raw[3 * nc:4 * nc], "u": raw[4 * nc:7 * nc].reshape(3, nc),
            "sums": raw[7 * nc:7 * nc + 5], "bad": int(raw[7 * nc + 5:].view(np.int64)[0])}


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_c_client_matches_binding_and_oracle(prec):
    if not os.path.exists(EXE):
        pytest.fail("tests/c_client/rlb_run is not built (run __graft_entry__.build())")
    import paper_1211_3286_amd as rlb
    prob = wl.random_modes(37, 29, 23, seed=12, umax=0.2, amp=0.1, tau_v=0.8, tau_e=0.55,
                           tau_eps=0.7, tau_f=0.63, bc=(1, 0, 0))
    T = 25
    d = tempfile.mkdtemp()
    c = _run_client(prob, prec, T, d)
    sim = rlb.from_problems(prob, precision=prec)
    sim.step(T)
    m = sim.moments()
    for k in ("n", "eps", "P", "gamma", "u"):
        assert np.array_equal(c[k], m[k].cpu().numpy()), k
    assert np.array_equal(c["sums"], m["sums"]) and c["bad"] == 0
    sim.close()
    F = oracle.run(prob, T).fields()
    err = {k: relmax(c[k], F[k].reshape(c[k].shape)) for k in ("n", "eps", "P", "gamma", "u")}
    say("  c client vs oracle", err)
    assert max(err.values()) < TOL[prec], err
