"""Oracle pins: the FP64 adjoint against central finite differences.

The adjoint differentiates L = sum(|u(T) - u_t|^2 + (eps(T) - eps_t)^2) with
respect to (tau_v, tau_e, tau_eps) and the initial fields. Finite differences
of the forward oracle are the independent check (derivative definition).
"""

import copy

import numpy as np
import pytest

import workloads as wl


def _loss(orc, prob, T, ut, et):
    F = orc.run(prob, T).fields()
    return float(((F["u"] - ut) ** 2).sum() + ((F["eps"] - et) ** 2).sum()), F


def _with(prob, **kw):
    q = copy.deepcopy(prob)
    for k, v in kw.items():
        setattr(q.params, k, v)
    return q


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 0)])
def test_adjoint_matches_fd(orc, bc):
    prob = wl.random_modes(6, 5, 1, seed=9, umax=0.15, amp=0.1, tau_v=0.8, tau_e=0.6,
                           tau_eps=0.7, tau_f=0.8, bc=bc)
    T = 12
    rng = np.random.default_rng(4)
    ut = prob.u + 0.01 * rng.normal(size=prob.u.shape)
    et = prob.eps + 0.01 * rng.normal(size=prob.eps.shape)
    L0, F = _loss(orc, prob, T, ut, et)
    dtau, de0, du0 = orc.grad(prob, T, 2 * (F["u"] - ut), 2 * (F["eps"] - et))
    h = 1e-4
    for i, name in enumerate(("tau_v", "tau_e", "tau_eps")):
        t0 = getattr(prob.params, name)
        lp, _ = _loss(orc, _with(prob, **{name: t0 + h}), T, ut, et)
        lm, _ = _loss(orc, _with(prob, **{name: t0 - h}), T, ut, et)
        fd = (lp - lm) / (2 * h)
        assert abs(dtau[i] - fd) < 1e-6 * max(abs(fd), np.abs(dtau).max())
    for cell in [(0, 0, 0), (0, 3, 2), (0, 4, 5)]:
        q = copy.deepcopy(prob)
        q.eps[cell] += h
        lp, _ = _loss(orc, q, T, ut, et)
        q.eps[cell] -= 2 * h
        lm, _ = _loss(orc, q, T, ut, et)
        fd = (lp - lm) / (2 * h)
        assert abs(de0[cell] - fd) < 1e-6 * max(abs(fd), np.abs(de0).max())
        for c in range(2):
            q = copy.deepcopy(prob)
            q.u[(c,) + cell] += h
            lp, _ = _loss(orc, q, T, ut, et)
            q.u[(c,) + cell] -= 2 * h
            lm, _ = _loss(orc, q, T, ut, et)
            fd = (lp - lm) / (2 * h)
            assert abs(du0[(c,) + cell] - fd) < 1e-6 * max(abs(fd), np.abs(du0).max())


def test_adjoint_zero_steps_is_init_jacobian(orc):
    """T = 0: the gradient is the derivative of the recovery of g_eq(eps0, u0),
    i.e. the identity on (eps, u)."""
    prob = wl.random_modes(4, 3, 1, seed=2, umax=0.2)
    rng = np.random.default_rng(1)
    du = rng.normal(size=prob.u.shape)
    de = rng.normal(size=prob.eps.shape)
    dtau, de0, du0 = orc.grad(prob, 0, du, de)
    assert np.abs(dtau).max() == 0.0
    assert np.abs(de0 - de).max() < 1e-12
    assert np.abs(du0 - du).max() < 1e-12
