"""Oracle pins: the per-cell collision (Eqs. 5, 6, 30, 31, 35)."""

import numpy as np
import pytest

from workloads import Params


def _neq_state(orc, rng, amp=0.02):
    """A pre-collision state: equilibrium of a random field plus a perturbation."""
    u = rng.uniform(-0.3, 0.3, 3)
    eps = rng.uniform(0.5, 3.0)
    n = rng.uniform(0.5, 2.0)
    gam = 1.0 / np.sqrt(1.0 - u @ u)
    f = orc.feq(n, gam, u) * (1.0 + amp * rng.normal(size=19))
    g = orc.geq(eps, eps / 3.0, u) * (1.0 + amp * rng.normal(size=19))
    return f, g


def _fields(orc, f, g):
    e = orc.tables()["e"].astype(float)
    ok, F = orc.recover(f.sum(), g.sum(), e.T @ g)
    assert ok
    return F


def test_mrt_equals_bgk_when_rates_equal(orc):
    """All non-conserved rates 1/tau turn Eq. (30) into the BGK Eq. (6)."""
    rng = np.random.default_rng(20)
    for tau in (0.51, 0.8, 1.7, 15.5):
        p = Params(1, 1, 1, tau_f=0.9, tau_v=tau, tau_e=tau, tau_eps=tau, tau_q=tau)
        for _ in range(10):
            f, g = _neq_state(orc, rng)
            ok, fo, go = orc.collide_cell(p, f, g)
            assert ok
            F = _fields(orc, f, g)
            geq = orc.geq(F["eps"], F["P"], [F["ux"], F["uy"], F["uz"]])
            bgk = g - (g - geq) / tau
            assert np.abs(go - bgk).max() < 1e-14 * np.abs(g).max()


def test_f_is_bgk(orc):
    """Eq. (5): f* = f - (f - f_eq)/tau_f with f_eq of the recovered n, u."""
    rng = np.random.default_rng(21)
    p = Params(1, 1, 1, tau_f=0.63, tau_v=0.8, tau_e=0.55, tau_eps=0.7)
    for _ in range(10):
        f, g = _neq_state(orc, rng)
        ok, fo, go = orc.collide_cell(p, f, g)
        F = _fields(orc, f, g)
        feq = orc.feq(F["n"], F["gamma"], [F["ux"], F["uy"], F["uz"]])
        assert np.abs(fo - (f - (f - feq) / 0.63)).max() < 1e-14 * np.abs(f).max()


def test_collision_conserves(orc):
    """n gamma, sigma - P and sigma u are collision invariants (Eqs. 2-4)."""
    e = orc.tables()["e"].astype(float)
    rng = np.random.default_rng(22)
    p = Params(1, 1, 1, tau_f=0.7, tau_v=1.3, tau_e=0.52, tau_eps=0.9, tau_q=1.1)
    for _ in range(20):
        f, g = _neq_state(orc, rng, amp=0.1)
        ok, fo, go = orc.collide_cell(p, f, g)
        s = np.abs(g).sum()
        assert abs(fo.sum() - f.sum()) < 1e-14 * np.abs(f).sum()
        assert abs(go.sum() - g.sum()) < 1e-14 * s
        assert np.abs(e.T @ go - e.T @ g).max() < 1e-14 * s


def test_equilibrium_is_fixed_point(orc):
    rng = np.random.default_rng(23)
    p = Params(1, 1, 1, tau_f=0.7, tau_v=1.3, tau_e=0.52, tau_eps=0.9)
    for _ in range(10):
        f, g = _neq_state(orc, rng, amp=0.0)
        ok, fo, go = orc.collide_cell(p, f, g)
        assert np.abs(go - g).max() < 1e-14 * np.abs(g).max()
        assert np.abs(fo - f).max() < 1e-14 * np.abs(f).max()


@pytest.mark.parametrize("row,name", [(1, "tau_e"), (2, "tau_eps"), (4, "tau_q"), (9, "tau_v"),
                                      (10, "tau_q"), (11, "tau_v"), (12, "tau_q"),
                                      (13, "tau_v"), (14, "tau_v"), (15, "tau_v"),
                                      (16, "tau_q"), (18, "tau_q")])
def test_each_moment_relaxes_with_its_own_rate(orc, row, name):
    """Eqs. (31), (35): a deviation in one non-conserved moment k relaxes as
    (m_k - m_eq,k) -> (1 - 1/tau_k)(m_k - m_eq,k), leaving the others alone.
    tau_e is the bulk (energy) row, tau_v the shear rows, tau_q the ghosts."""
    t = orc.tables()
    M, Minv = t["M"], t["Minv"]
    taus = dict(tau_v=0.83, tau_e=0.57, tau_eps=1.21, tau_q=1.37)
    p = Params(1, 1, 1, tau_f=0.9, **taus)
    u = np.array([0.11, -0.07, 0.05])
    eps = 1.3
    geq = orc.geq(eps, eps / 3.0, u)
    dm = np.zeros(19)
    dm[row] = 1e-3 * np.abs(M[row] @ geq + 1.0)
    g = geq + Minv @ dm  # moments 0, 3, 5, 7 untouched -> same recovered fields
    f = orc.feq(1.0, 1.0 / np.sqrt(1 - u @ u), u)
    ok, fo, go = orc.collide_cell(p, f, g)
    dm_out = M @ go - M @ geq
    want = np.zeros(19)
    want[row] = (1.0 - 1.0 / taus[name]) * dm[row]
    assert np.abs(dm_out - want).max() < 1e-12 * np.abs(M @ geq).max()


def test_inadmissible_cell_is_left_alone(orc):
    p = Params(1, 1, 1)
    f = np.ones(19)
    g = -np.ones(19)  # E < 0
    ok, fo, go = orc.collide_cell(p, f, g)
    assert not ok
    assert np.array_equal(fo, f) and np.array_equal(go, g)
