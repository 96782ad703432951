"""Oracle pins: equilibria (Eqs. 7-9) against their moment constraints.

Eq. (10) and the text after Eq. (10): sum f_eq = n gamma, sum e f_eq = n gamma u.
Eqs. (A5)-(A6): sum g_eq = sigma - P, sum e g_eq = sigma u,
sum e e g_eq = sigma u u + P I (the ideal T^{ij} of Eq. 1).
Eq. (A7) as printed lacks a factor c_s^2 (compare Eq. A16, which uses it);
the corrected third moment is c_s^2 sigma (u_k d_ij + u_i d_jk + u_j d_ik).
"""

import numpy as np
import pytest

CS2 = 1.0 / 3.0


def _states(seed, n=40, umax=0.8):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        u = rng.normal(size=3)
        u *= rng.uniform(0.0, umax) / np.linalg.norm(u)
        yield rng.uniform(0.1, 4.0), rng.uniform(0.1, 10.0), u


def test_feq_moments(orc):
    e = orc.tables()["e"].astype(float)
    for n, eps, u in _states(1):
        gam = 1.0 / np.sqrt(1.0 - u @ u)
        f = orc.feq(n, gam, u)
        assert abs(f.sum() - n * gam) < 1e-14 * n * gam
        assert np.abs(e.T @ f - n * gam * u).max() < 1e-14 * n * gam
        # second moment of f_eq (used in Eq. 20): n gamma (u u + c_s^2 I)
        assert np.abs(np.einsum("a,ai,aj->ij", f, e, e)
                      - n * gam * (np.outer(u, u) + CS2 * np.eye(3))).max() < 1e-14 * n * gam


def test_geq_moments(orc):
    e = orc.tables()["e"].astype(float)
    for n, eps, u in _states(2):
        P = eps / 3.0
        sigma = (eps + P) / (1.0 - u @ u)
        g = orc.geq(eps, P, u)
        tol = 1e-14 * sigma
        assert abs(g.sum() - (sigma - P)) < tol                         # (A5)
        assert np.abs(e.T @ g - sigma * u).max() < tol                  # (A5)
        T2 = np.einsum("a,ai,aj->ij", g, e, e)
        assert np.abs(T2 - (sigma * np.outer(u, u) + P * np.eye(3))).max() < tol  # (A6)
        T3 = np.einsum("a,ai,aj,ak->ijk", g, e, e, e)
        d = np.eye(3)
        ref = CS2 * sigma * (np.einsum("k,ij->ijk", u, d) + np.einsum("i,jk->ijk", u, d)
                             + np.einsum("j,ik->ijk", u, d))
        assert np.abs(T3 - ref).max() < tol                             # (A7), corrected


def test_geq_general_pressure(orc):
    """Eqs. (8)-(9) hold the moment constraints for any P, not only P = eps/3."""
    e = orc.tables()["e"].astype(float)
    rng = np.random.default_rng(3)
    for _ in range(20):
        u = rng.uniform(-0.3, 0.3, 3)
        eps = rng.uniform(0.5, 2.0)
        P = rng.uniform(0.05, 1.0)
        sigma = (eps + P) / (1.0 - u @ u)
        g = orc.geq(eps, P, u)
        assert abs(g.sum() - (sigma - P)) < 1e-14 * sigma
        T2 = np.einsum("a,ai,aj->ij", g, e, e)
        assert np.abs(T2 - (sigma * np.outer(u, u) + P * np.eye(3))).max() < 1e-14 * sigma


def test_rest_state_values(orc):
    """At u = 0 and P = eps/3 (sigma = 4P): g_0 = P, faces P/6, edges P/12."""
    e = orc.tables()["e"]
    r2 = (e * e).sum(axis=1)
    for P in (0.1, 1.0, 7.5):
        g = orc.geq(3 * P, P, np.zeros(3))
        assert abs(g[0] - P) < 1e-15 * P
        assert np.abs(g[r2 == 1] - P / 6).max() < 1e-15 * P
        assert np.abs(g[r2 == 2] - P / 12).max() < 1e-15 * P
        f = orc.feq(2.0, 1.0, np.zeros(3))
        assert np.allclose(f, 2.0 * orc.tables()["w"], rtol=1e-15, atol=0)


def test_geq_reduces_to_standard_lb_form(orc):
    """With P = c_s^2 sigma the g_eq of Eqs. (8)-(9) equals the standard form
    w sigma (1 + e.u/c_s^2 + (e.u)^2/(2 c_s^4) - u^2/(2 c_s^2)) plus the
    rest-population shift that moves sum g from sigma to sigma - P (Eq. 27)."""
    t = orc.tables()
    e, w = t["e"].astype(float), t["w"]
    rng = np.random.default_rng(4)
    for _ in range(10):
        u = rng.uniform(-0.2, 0.2, 3)
        sigma = rng.uniform(0.5, 3.0)
        P = CS2 * sigma
        eps = sigma * (1.0 - u @ u) - P
        g = orc.geq(eps, P, u)
        eu = e @ u
        ghat = w * sigma * (1 + eu / CS2 + eu ** 2 / (2 * CS2 ** 2) - (u @ u) / (2 * CS2))
        ghat[0] -= P
        assert np.abs(g - ghat).max() < 1e-14 * sigma
