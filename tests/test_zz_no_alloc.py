"""GPU test of rlb_run_noalloc, the allocation-free run of include/rlb.h.

Its output must equal that of the handle path (rlb_init + rlb_step +
rlb_moments) on the same inputs, to the parity bar (FP64 1e-12, FP32 1e-5,
max-norm relative), over a sequence of calls on one device, each lattice
smaller than the one before, so that every call reuses the fixed scratch
array the previous one left behind. The first case leaves inadmissible cells
(a strong blast), so the next call also checks that the counters are cleared
between calls. Called through the C ABI (ctypes) with device fields.
"""

import numpy as np
import pytest

import workloads as wl
from gpu_helpers import say

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


def _modes(dims, bc=(0, 0, 0)):
    prob = wl.random_modes(*dims, seed=5, umax=0.2, amp=0.1, tau_v=0.8, tau_e=0.55,
                           tau_eps=0.7, tau_f=0.8, bc=bc)
    return prob


def _d2q9_c7(nx, ny):
    prob = wl.random_modes(nx, ny, 1, seed=11, umax=0.2, amp=0.1, tau_v=1.3, tau_e=0.6,
                           tau_eps=0.7, tau_f=0.7, bc=(0, 1, 0))
    prob.params.lattice = "d2q9"
    prob.params.correction = 1
    return prob


# (name, problem, precision, steps, tolerance); cells decrease down the list
CASES = [
    ("blast 32^3 FP64, zero-gradient faces", lambda: wl.blast(32), FP64, 20, 1e-12),
    ("random modes 40x30x20 FP64, mixed faces", lambda: _modes((40, 30, 20), bc=(0, 1, 0)),
     FP64, 25, 1e-12),
    ("random modes 13x11x7 FP32, periodic", lambda: _modes((13, 11, 7)), FP32, 25, 1e-5),
    ("D2Q9 + correction 29x23 FP64", lambda: _d2q9_c7(29, 23), FP64, 15, 1e-12),
]


def _rel(a, b):
    """max-norm relative difference; inadmissible cells (NaN fields) must be
    NaN on both sides."""
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    na, nb = np.isnan(a), np.isnan(b)
    assert np.array_equal(na, nb)
    a, b = a[~na], b[~nb]
    if b.size == 0:
        return 0.0
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_noalloc_equals_the_handle_path():
    import torch
    import paper_1211_3286_amd as rlb
    torch.cuda.set_device(0)
    prev_cells = None
    bads = []
    for name, make, prec, steps, tol in CASES:
        prob = make()
        p = prob.params
        assert prev_cells is None or p.ncells < prev_cells
        prev_cells = p.ncells
        say(f"noalloc case: {name}, {p.ncells} cells, {steps} steps")
        n0 = torch.from_numpy(np.ascontiguousarray(prob.n.ravel())).cuda()
        e0 = torch.from_numpy(np.ascontiguousarray(prob.eps.ravel())).cuda()
        u0 = torch.from_numpy(np.ascontiguousarray(prob.u.reshape(3, -1))).cuda()
        lattice = getattr(p, "lattice", "d3q19")
        corr = int(getattr(p, "correction", 0))
        got = rlb.run_noalloc(p, n0, e0, u0, steps, precision=prec, lattice=lattice,
                              correction=corr, allow_unphysical=True)
        sim = rlb.Simulation([p], n0, e0, u0, precision=prec, lattice=lattice, correction=corr)
        sim.step(steps)
        ref = sim.moments(allow_unphysical=True)
        kernel = sim.kernel_name
        sim.close()
        errs = {k: _rel(got[k], ref[k]) for k in ("n", "eps", "P", "gamma", "u")}
        errs["sums"] = float(np.abs(got["sums"] - ref["sums"]).max() / np.abs(ref["sums"][:2]).max())
        say(f"  vs handle path ({kernel}): {errs}; inadmissible {got['bad']} / {ref['bad']}")
        # after the blast the shared array holds its counts: equal counts
        # here mean the call started from zero
        assert got["bad"] == ref["bad"]
        for k, v in errs.items():
            assert v <= tol, (name, k, v)
        bads.append(got["bad"])
    assert bads[0] > 0 and not any(bads[1:])


def test_noalloc_repeated_call_is_identical():
    """Two identical calls in a row give bit-identical outputs: nothing of the
    first call's scratch contents leaks into the second."""
    import torch
    import paper_1211_3286_amd as rlb
    prob = _modes((24, 20, 16))
    p = prob.params
    say(f"noalloc repeat: random modes 24x20x16 FP32, {p.ncells} cells, 12 steps, twice")
    n0 = torch.from_numpy(np.ascontiguousarray(prob.n.ravel())).cuda()
    e0 = torch.from_numpy(np.ascontiguousarray(prob.eps.ravel())).cuda()
    u0 = torch.from_numpy(np.ascontiguousarray(prob.u.reshape(3, -1))).cuda()
    a = rlb.run_noalloc(p, n0, e0, u0, 12, precision=FP32)
    b = rlb.run_noalloc(p, n0, e0, u0, 12, precision=FP32)
    for k in ("n", "eps", "P", "gamma", "u"):
        assert torch.equal(a[k], b[k]), k
    assert np.array_equal(a["sums"], b["sums"]) and a["bad"] == b["bad"] == 0


def test_noalloc_refuses_what_does_not_fit():
    """A lattice beyond the fixed array is refused with RLB_E_SCRATCH, and the
    next call on the device still works."""
    import torch
    import paper_1211_3286_amd as rlb
    big = wl.uniform(64, 64, 64)
    nc = big.params.ncells
    say(f"noalloc refusal: 64^3 FP64 ({nc} cells)")
    n0 = torch.ones(nc, dtype=torch.float64, device="cuda")
    u0 = torch.zeros(3, nc, dtype=torch.float64, device="cuda")
    with pytest.raises(rlb.RLBError) as ei:
        rlb.run_noalloc(big.params, n0, n0, u0, 1, precision=FP64)
    assert ei.value.code == -8
    small = _modes((9, 8, 7))
    n1 = torch.from_numpy(np.ascontiguousarray(small.n.ravel())).cuda()
    e1 = torch.from_numpy(np.ascontiguousarray(small.eps.ravel())).cuda()
    u1 = torch.from_numpy(np.ascontiguousarray(small.u.reshape(3, -1))).cuda()
    out = rlb.run_noalloc(small.params, n1, e1, u1, 3, precision=FP64)
    assert out["bad"] == 0 and np.isfinite(out["sums"]).all()
