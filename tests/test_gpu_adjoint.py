"""GPU parity of the hand-written adjoint (rlb_grad) and the autograd wrapper.

* FP64 adjoint vs the oracle's FP64 complex-step adjoint, element by element,
  for random cotangents (dL/du, dL/deps) on lattices with periodic, clamped and
  mixed ends and with partial checkpoint segments: <= 1e-10 (max-norm rel.).
* FP32 adjoint vs the oracle on a 64 x 64 periodic field: <= 1e-4.
* FP32 adjoint vs central finite differences (h = 1e-4) of the FP64 forward:
  within 1e-4 of max(|FD|, |grad|) per component, including the full
  512 x 512 x 1000-step shear-wave/vortex case with checkpoints every 50.
"""

import copy

import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_helpers import relmax, say

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


def _gpu_grad(prob, T, K, prec, du, de):
    import torch
    import paper_1211_3286_amd as rlb
    sim = rlb.from_problems(prob, precision=prec, ckpt_every=K, tape_steps=max(T, 1))
    if T:
        sim.step(T)
    nc = prob.params.ncells
    dtau, de0, du0 = sim.grad(torch.from_numpy(du.reshape(3, nc)),
                              torch.from_numpy(de.reshape(nc)))
    out = (dtau, de0.cpu().numpy().reshape(prob.eps.shape),
           du0.cpu().numpy().reshape(prob.u.shape))
    sim.close()
    return out


def _cotangents(prob, seed=5):
    rng = np.random.default_rng(seed)
    return rng.normal(size=prob.u.shape), rng.normal(size=prob.eps.shape)


CASES = [
    # (nx, ny, nz, bc, T, K, tau_q)
    (8, 6, 1, (0, 0, 0), 13, 5, 0.0),
    (6, 5, 4, (1, 1, 1), 9, 4, 0.0),
    (12, 1, 10, (0, 0, 1), 10, 10, 1.3),
    (5, 7, 3, (1, 0, 1), 7, 3, 0.0),
    (9, 4, 2, (0, 1, 0), 0, 4, 0.0),
    # planar lattices: rows longer than one 64-cell wave with a ragged last
    # wave, clamped and periodic axes, a last partial segment (T = 11, K = 4;
    # T = 9, K = 5) and a single segment with nothing recomputed beside the
    # reverse steps (T = K)
    (70, 37, 1, (1, 0, 0), 11, 4, 0.0),
    (33, 16, 1, (0, 1, 1), 9, 5, 0.0),
    (31, 15, 1, (1, 1, 0), 8, 8, 0.0),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}_bc{c[3]}_T{c[4]}K{c[5]}")
def test_fp64_adjoint_matches_oracle(case):
    nx, ny, nz, bc, T, K, tq = case
    prob = wl.random_modes(nx, ny, nz, seed=11, umax=0.2, amp=0.1, tau_v=0.8, tau_e=0.6,
                           tau_eps=0.7, tau_f=0.8, bc=bc)
    prob.params.tau_q = tq
    du, de = _cotangents(prob)
    say("adjoint fp64", case)
    g_tau, g_e0, g_u0 = _gpu_grad(prob, T, K, FP64, du, de)
    o_tau, o_e0, o_u0 = oracle.grad(prob, T, du, de)
    say("  tau gpu", g_tau, "oracle", o_tau)
    assert relmax(g_tau, o_tau) < 1e-10
    assert relmax(g_e0, o_e0) < 1e-10
    assert relmax(g_u0, o_u0) < 1e-10


def test_fp64_adjoint_matches_oracle_two_layers_of_row_blocks():
    """520 x 520 rows of 2 cells: 67,600 blocks of 4 rows exceed the 65,535 a
    grid's y holds, so the launches take two z layers of row blocks (131,070
    blocks, not a multiple of the 8 XCDs, the second layer mostly past the
    last row). Every cell must still be taken exactly once by the kernels'
    block renumbering."""
    prob = wl.random_modes(2, 520, 520, seed=11, umax=0.2, amp=0.1, tau_v=0.8, tau_e=0.6,
                           tau_eps=0.7, tau_f=0.8, bc=(0, 1, 0))
    du, de = _cotangents(prob)
    say("adjoint fp64 2x520x520 T3 K2 (two z layers of row blocks)")
    g_tau, g_e0, g_u0 = _gpu_grad(prob, 3, 2, FP64, du, de)
    o_tau, o_e0, o_u0 = oracle.grad(prob, 3, du, de)
    say("  tau gpu", g_tau, "oracle", o_tau)
    assert relmax(g_tau, o_tau) < 1e-10
    assert relmax(g_e0, o_e0) < 1e-10
    assert relmax(g_u0, o_u0) < 1e-10


def test_fp32_adjoint_matches_oracle_64x64():
    prob = wl.shear_vortex(64, seed=1212)
    T, K = 100, 50
    du, de = _cotangents(prob, seed=6)
    g_tau, g_e0, g_u0 = _gpu_grad(prob, T, K, FP32, du, de)
    o_tau, o_e0, o_u0 = oracle.grad(prob, T, du, de)
    err = (relmax(g_tau, o_tau), relmax(g_e0, o_e0), relmax(g_u0, o_u0))
    say("adjoint fp32 64x64 vs oracle: tau", g_tau, o_tau, "errors", err)
    assert max(err) < 1e-4


def _loss_fp64(prob, T, ut, et):
    import torch
    import paper_1211_3286_amd as rlb
    sim = rlb.from_problems(prob, precision=FP64)
    sim.step(T)
    m = sim.moments()
    u = m["u"].cpu().numpy().reshape(prob.u.shape)
    e = m["eps"].cpu().numpy().reshape(prob.eps.shape)
    sim.close()
    return float(((u - ut) ** 2).sum() + ((e - et) ** 2).sum()), u, e


def _with_tau(prob, **kw):
    q = copy.deepcopy(prob)
    for k, v in kw.items():
        setattr(q.params, k, v)
    return q


def _target(prob, T, seed):
    """Same model at perturbed relaxation times, plus 1 % noise."""
    tv, te, tpe = wl.perturbed_taus((prob.params.tau_v, prob.params.tau_e,
                                     prob.params.tau_eps), seed=seed)
    _, ut, et = _loss_fp64(_with_tau(prob, tau_v=tv, tau_e=te, tau_eps=tpe), T, 0.0, 0.0)
    z = wl.target_noise(prob.eps.shape, seed=seed)
    ut = ut + 0.01 * np.sqrt((ut ** 2).mean()) * z[:3]
    et = et + 0.01 * np.sqrt((et ** 2).mean()) * z[3]
    return ut, et


def _check_fd(prob, T, K, cells, seed):
    ut, et = _target(prob, T, seed)
    L0, u, e = _loss_fp64(prob, T, ut, et)
    du, de = 2.0 * (u - ut), 2.0 * (e - et)
    g_tau, g_e0, g_u0 = _gpu_grad(prob, T, K, FP32, du, de)
    h = 1e-4
    fd = []
    for name in ("tau_v", "tau_e", "tau_eps"):
        t0 = getattr(prob.params, name)
        lp = _loss_fp64(_with_tau(prob, **{name: t0 + h}), T, ut, et)[0]
        lm = _loss_fp64(_with_tau(prob, **{name: t0 - h}), T, ut, et)[0]
        fd.append((lp - lm) / (2 * h))
    fd = np.array(fd)
    say("dL/dtau adjoint", g_tau, "fd", fd)
    scale = max(np.abs(fd).max(), np.abs(g_tau).max())
    assert np.abs(g_tau - fd).max() < 1e-4 * scale
    for cell in cells:
        q = copy.deepcopy(prob)
        q.eps[cell] += h
        lp = _loss_fp64(q, T, ut, et)[0]
        q.eps[cell] -= 2 * h
        lm = _loss_fp64(q, T, ut, et)[0]
        fde = (lp - lm) / (2 * h)
        q = copy.deepcopy(prob)
        q.u[(0,) + cell] += h
        lp = _loss_fp64(q, T, ut, et)[0]
        q.u[(0,) + cell] -= 2 * h
        lm = _loss_fp64(q, T, ut, et)[0]
        fdu = (lp - lm) / (2 * h)
        say("cell", cell, "deps0", g_e0[cell], fde, "dux0", g_u0[(0,) + cell], fdu)
        assert abs(g_e0[cell] - fde) < 1e-4 * max(abs(fde), np.abs(g_e0).max())
        assert abs(g_u0[(0,) + cell] - fdu) < 1e-4 * max(abs(fdu), np.abs(g_u0).max())


def test_fp32_adjoint_vs_finite_differences_32x32():
    prob = wl.shear_vortex(32, seed=1212)
    _check_fd(prob, 60, 25, [(0, 3, 7), (0, 20, 30)], seed=1212)


def test_fp32_adjoint_vs_finite_differences_full_512x512():
    """The full adjoint workload: 512 x 512 x 1, 1000 steps, checkpoints every 50."""
    prob = wl.shear_vortex(512, seed=1212)
    _check_fd(prob, 1000, 50, [(0, 100, 200)], seed=1212)


def test_autograd_function():
    import torch
    import paper_1211_3286_amd as rlb
    prob = wl.shear_vortex(24, seed=3)
    p = prob.params
    dev = torch.device("cuda")
    eps0 = torch.tensor(prob.eps, device=dev, requires_grad=True)
    u0 = torch.tensor(prob.u, device=dev, requires_grad=True)
    n0 = torch.tensor(prob.n, device=dev)
    tau = torch.tensor([p.tau_v, p.tau_e, p.tau_eps], dtype=torch.float64, requires_grad=True)
    u, e = rlb.RLBStep.apply(eps0, u0, n0, tau, p, 30, rlb.FP64, 8)
    loss = (u ** 2).sum() + (e ** 2).sum()
    loss.backward()
    du = 2.0 * u.detach().cpu().numpy()
    de = 2.0 * e.detach().cpu().numpy()
    o_tau, o_e0, o_u0 = oracle.grad(prob, 30, du, de)
    assert relmax(tau.grad.numpy(), o_tau) < 1e-10
    assert relmax(eps0.grad.cpu().numpy(), o_e0) < 1e-10
    assert relmax(u0.grad.cpu().numpy(), o_u0) < 1e-10


def test_grad_requires_tape():
    import torch
    import paper_1211_3286_amd as rlb
    prob = wl.shear_vortex(16)
    sim = rlb.from_problems(prob, precision=FP32)
    sim.step(2)
    with pytest.raises(rlb.RLBError) as ei:
        sim.grad(torch.zeros(3, 256, dtype=torch.float64), torch.zeros(256, dtype=torch.float64))
    assert ei.value.code == -6
    sim2 = rlb.from_problems(prob, precision=FP32, ckpt_every=4, tape_steps=8)
    sim2.step(9)  # beyond the tape
    with pytest.raises(rlb.RLBError) as ei:
        sim2.grad(torch.zeros(3, 256, dtype=torch.float64), torch.zeros(256, dtype=torch.float64))
    assert ei.value.code == -6
