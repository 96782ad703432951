"""GPU tests of C-ABI paths the Python wrapper does not take, and edge cases.

* Host-pointer I/O: rlb_init with host fields, rlb_moments / rlb_populations /
  rlb_grad writing host arrays (staged through the workspace).
* Degenerate lattices: 1 x 1 x 1 and 2 x 1 x 1, periodic and zero-gradient.
* A batch holding a one-cell member; diagnostics from segmented launches.
* Workspace and tau validation on a live device.
"""

import ctypes

import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_helpers import relmax, say

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


def _host_handle(problems, prec, **opt):
    import torch
    import paper_1211_3286_amd as rlb
    if not isinstance(problems, list):
        problems = [problems]
    n, e, u = rlb.problem_fields(problems)
    n = np.ascontiguousarray(n)
    e = np.ascontiguousarray(e)
    u = np.ascontiguousarray(u)
    arr = rlb.cparams([p.params for p in problems])
    o = rlb.options(prec, **opt)
    size = rlb.workspace_size([p.params for p in problems], o)
    ws = torch.empty(size + 256, dtype=torch.uint8, device="cuda")
    ptr = (ws.data_ptr() + 255) // 256 * 256
    h = ctypes.c_void_p(0)
    code = rlb.lib().rlb_init(ctypes.byref(h), arr, len(problems), ctypes.byref(o),
                              n.ctypes.data, e.ctypes.data, u.ctypes.data, 0, ptr, size, None)
    assert code == 0, rlb.status_string(code)
    return h, ws, sum(p.params.ncells for p in problems)


def _host_fields(h, nc):
    import paper_1211_3286_amd as rlb
    out = {k: np.zeros(nc) for k in ("n", "eps", "P", "gamma")}
    out["u"] = np.zeros((3, nc))
    sums = (ctypes.c_double * 5)()
    bad = ctypes.c_int64(-1)
    code = rlb.lib().rlb_moments(h, out["n"].ctypes.data, out["eps"].ctypes.data,
                                 out["P"].ctypes.data, out["gamma"].ctypes.data,
                                 out["u"].ctypes.data, sums, ctypes.byref(bad), 0)
    assert code == 0, rlb.status_string(code)
    f = np.zeros((19, nc))
    g = np.zeros((19, nc))
    assert rlb.lib().rlb_populations(h, f.ctypes.data, g.ctypes.data, 0) == 0
    return out, np.array(sums[:]), bad.value, f, g


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_host_pointer_paths(prec):
    import paper_1211_3286_amd as rlb
    prob = wl.random_modes(20, 9, 11, seed=8, umax=0.2, amp=0.1, bc=(0, 1, 0))
    h, ws, nc = _host_handle(prob, prec)
    assert rlb.lib().rlb_step(h, 9) == 0
    out, sums, bad, f, g = _host_fields(h, nc)
    st = oracle.run(prob, 9)
    F = st.fields()
    tol = 1e-12 if prec == FP64 else 1e-5
    assert bad == 0
    assert relmax(f.reshape(st.f.shape), st.f) < tol and relmax(g.reshape(st.g.shape), st.g) < tol
    assert relmax(out["eps"].reshape(F["eps"].shape), F["eps"]) < tol
    assert relmax(out["gamma"].reshape(F["gamma"].shape), F["gamma"]) < tol
    assert relmax(sums, F["sums"]) < (1e-13 if prec == FP64 else 1e-7)
    rlb.lib().rlb_free(h)


def test_host_pointer_grad():
    import paper_1211_3286_amd as rlb
    prob = wl.random_modes(7, 6, 5, seed=9, umax=0.15, amp=0.1, bc=(1, 0, 1))
    h, ws, nc = _host_handle(prob, FP64, ckpt_every=3, tape_steps=10)
    assert rlb.lib().rlb_step(h, 10) == 0
    rng = np.random.default_rng(2)
    du = rng.normal(size=(3, nc))
    de = rng.normal(size=nc)
    dtau = (ctypes.c_double * 3)()
    de0 = np.zeros(nc)
    du0 = np.zeros((3, nc))
    code = rlb.lib().rlb_grad(h, du.ctypes.data, de.ctypes.data, dtau, de0.ctypes.data,
                              du0.ctypes.data, 0)
    assert code == 0, rlb.status_string(code)
    o_tau, o_e0, o_u0 = oracle.grad(prob, 10, du.reshape(prob.u.shape),
                                    de.reshape(prob.eps.shape))
    assert relmax(np.array(dtau[:]), o_tau) < 1e-10
    assert relmax(de0.reshape(o_e0.shape), o_e0) < 1e-10
    assert relmax(du0.reshape(o_u0.shape), o_u0) < 1e-10
    rlb.lib().rlb_free(h)


@pytest.mark.parametrize("dims,bc", [((1, 1, 1), (0, 0, 0)), ((1, 1, 1), (1, 1, 1)),
                                     ((2, 1, 1), (0, 0, 0)), ((2, 1, 1), (1, 0, 1)),
                                     ((1, 3, 1), (1, 1, 1))])
def test_degenerate_lattices(dims, bc):
    import paper_1211_3286_amd as rlb
    prob = wl.random_modes(*dims, seed=4, umax=0.3, amp=0.2, bc=bc)
    sim = rlb.from_problems(prob, precision=FP64)
    sim.step(17)
    f, g = [t.cpu().numpy() for t in sim.populations()]
    st = oracle.run(prob, 17)
    say("degenerate", dims, bc, sim.kernel_name)
    assert relmax(f.reshape(st.f.shape), st.f) < 1e-12
    assert relmax(g.reshape(st.g.shape), st.g) < 1e-12


def test_batch_with_one_cell_member_and_segment_diagnostics():
    import paper_1211_3286_amd as rlb
    members = [wl.random_modes(1, 1, 1, seed=1, umax=0.1),
               wl.tube_batch(n_tubes=1, seed=11, lmin=700, lmax=700)[0],
               wl.random_modes(6, 5, 30, seed=2, umax=0.2, amp=0.1, bc=(0, 0, 1))]
    names = None
    ref_sums = None
    for v in range(len(rlb.from_problems(members, precision=FP64).variants())):
        sim = rlb.from_problems(members, precision=FP64, diag_every=1)
        names = sim.variants()
        sim.variant = v
        try:
            sim.step(5)
        except rlb.RLBError as e:  # tube rounds need a batch of 1 x 1 x L members
            assert e.code == -7 and "tubes" in names[v]
            continue
        sums, step, bad = sim.diagnostics()
        assert step == 5 and bad == 0
        if ref_sums is None:
            # the diagnostics of step 5 sum the populations streamed into it;
            # collision conserves N, E, M, so they equal the sums of state 5
            ref_sums = np.zeros(5)
            for p in members:
                ref_sums += oracle.run(p, 5).fields()["sums"]
        assert relmax(sums, ref_sums) < 1e-13, names[v]
        f, g = [t.cpu().numpy() for t in sim.populations()]
        off = 0
        for p in members:
            st = oracle.run(p, 5)
            nc = p.params.ncells
            assert relmax(f[:, off:off + nc].reshape(st.f.shape), st.f) < 1e-12, names[v]
            off += nc


def test_validation_on_device():
    import torch
    import paper_1211_3286_amd as rlb
    prob = wl.random_modes(8, 8, 8, seed=1)
    with pytest.raises(rlb.RLBError) as ei:
        bad = wl.random_modes(8, 8, 8, seed=1)
        bad.params.tau_e = 0.5
        rlb.from_problems(bad)
    assert ei.value.code == -2
    with pytest.raises(rlb.RLBError) as ei:
        bad = wl.random_modes(8, 8, 8, seed=1)
        bad.eps[3, 2, 1] = -1.0
        rlb.from_problems(bad)  # device fields: validated by a kernel
    assert ei.value.code == -3
    with pytest.raises(rlb.RLBError) as ei:
        bad = wl.random_modes(8, 8, 8, seed=1)
        bad.u[0, 1, 1, 1] = 1.0
        rlb.from_problems(bad)
    assert ei.value.code == -3
    sim = rlb.from_problems(prob)
    assert sim.steps == 0
    with pytest.raises(rlb.RLBError):
        sim.variant = 99
    sim.step(0)
    assert sim.steps == 0
