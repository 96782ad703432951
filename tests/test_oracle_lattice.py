"""Oracle pins: D3Q19 lattice, moment basis and the printed D2Q9 Eq. (34).

Each check compares the oracle's tables with something the paper or plain
mathematics fixes, never with a retyped copy of the oracle's own formulas.
"""

import itertools
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_velocity_set_is_d3q19(orc):
    t = orc.tables()
    e = t["e"]
    # rest + 6 faces + 12 edges, every vector distinct, opposite pairs present
    r2 = (e * e).sum(axis=1)
    assert sorted(r2.tolist()) == [0] + [1] * 6 + [2] * 12
    assert len({tuple(v) for v in e.tolist()}) == 19
    for v in e.tolist():
        assert [-c for c in v] in e.tolist()
    assert np.abs(e).max() == 1


def test_weights_isotropy(orc):
    """sum w = 1; sum w e_i e_j = cs^2 delta; sum w e_i e_j e_k e_l = cs^4 (dd + dd + dd).

    These are the lattice conditions behind Eqs. (7)-(10) with c_s^2 = 1/3.
    """
    t = orc.tables()
    e = t["e"].astype(float)
    w = t["w"]
    assert np.allclose(w * 36, np.round(w * 36), atol=0, rtol=1e-15)
    assert abs(w.sum() - 1.0) < 1e-15
    d = np.eye(3)
    cs2 = 1.0 / 3.0
    assert np.abs(np.einsum("a,ai->i", w, e)).max() < 1e-16
    assert np.abs(np.einsum("a,ai,aj->ij", w, e, e) - cs2 * d).max() < 1e-15
    assert np.abs(np.einsum("a,ai,aj,ak->ijk", w, e, e, e)).max() < 1e-16
    t4 = np.einsum("a,ai,aj,ak,al->ijkl", w, e, e, e, e)
    ref = cs2 ** 2 * (np.einsum("ij,kl->ijkl", d, d) + np.einsum("ik,jl->ijkl", d, d)
                      + np.einsum("il,jk->ijkl", d, d))
    assert np.abs(t4 - ref).max() < 1e-15


def test_basis_orthogonal_and_invertible(orc):
    t = orc.tables()
    M, Minv = t["M"], t["Minv"]
    G = M @ M.T
    assert np.abs(G - np.diag(np.diag(G))).max() == 0.0
    assert np.allclose(np.diag(G), t["norms"], rtol=0, atol=0)
    assert np.linalg.matrix_rank(M) == 19
    assert np.abs(Minv @ M - np.eye(19)).max() < 1e-14
    assert np.abs(M @ Minv - np.eye(19)).max() < 1e-14
    # Orthogonality makes the inverse M^T diag(1/|row|^2).
    assert np.abs(Minv - M.T / t["norms"][None, :]).max() < 1e-15


def test_conserved_rows_are_eq10_moments(orc):
    """Rows 0, 3, 5, 7 are 1, e_x, e_y, e_z: the sums of Eq. (10)."""
    t = orc.tables()
    M, e = t["M"], t["e"]
    assert np.all(M[0] == 1)
    for row, axis in ((3, 0), (5, 1), (7, 2)):
        assert np.all(M[row] == e[:, axis])


def _rand_state(rng):
    u = rng.uniform(-0.5, 0.5, 3)
    u *= rng.uniform(0.0, 0.7) / max(np.linalg.norm(u), 1e-12)
    eps = rng.uniform(0.2, 5.0)
    P = eps / 3.0
    gam2 = 1.0 / (1.0 - u @ u)
    return eps, P, u, (eps + P) * gam2


def test_d2q9_eq34_golden(orc):
    """M_D2Q9 g_eq(Eqs. 32-33) equals the printed Eq. (34) for random states."""
    coef = np.loadtxt(os.path.join(GOLDEN, "eq34_d2q9_meq.txt"))
    t = orc.d2q9_tables()
    rng = np.random.default_rng(34)
    for _ in range(50):
        u = rng.uniform(-0.4, 0.4, 2)
        sigma = rng.uniform(0.5, 3.0)
        P = rng.uniform(0.05, 0.5) * sigma
        geq = orc.d2q9_geq(sigma, P, u)
        m = t["M"] @ geq
        basis = np.array([sigma, sigma * (u @ u), P, sigma * u[0], sigma * u[1],
                          sigma * (u[0] ** 2 - u[1] ** 2), sigma * u[0] * u[1]])
        assert np.abs(m - coef @ basis).max() < 1e-13 * sigma


def test_d2q9_basis_orthogonal(orc):
    M = orc.d2q9_tables()["M"]
    G = M @ M.T
    assert np.abs(G - np.diag(np.diag(G))).max() == 0.0


def test_d3q19_moment_equilibria_from_A5_A6(orc):
    """Rows of M g_eq that Eqs. (A5)-(A6) fix.

    rho: sigma - P; j: sigma u (A5); 3p_xx = sum (3 e_x^2 - e^2) g_eq,
    p_ww = sum (e_y^2 - e_z^2) g_eq, p_ij = sum e_i e_j g_eq (A6); the energy
    row 19 e^2 - 30 combines the trace of (A6) with (A5).
    """
    t = orc.tables()
    M = t["M"]
    rng = np.random.default_rng(6)
    for _ in range(50):
        eps, P, u, sigma = _rand_state(rng)
        m = M @ orc.geq(eps, P, u)
        Pi = sigma * np.outer(u, u) + P * np.eye(3)  # (A6)
        tol = 1e-13 * sigma
        assert abs(m[0] - (sigma - P)) < tol
        assert np.abs(m[[3, 5, 7]] - sigma * u).max() < tol
        assert abs(m[1] - (19 * np.trace(Pi) - 30 * (sigma - P))) < 30 * tol
        assert abs(m[9] - (3 * Pi[0, 0] - np.trace(Pi))) < tol
        assert abs(m[11] - (Pi[1, 1] - Pi[2, 2])) < tol
        assert abs(m[13] - Pi[0, 1]) < tol
        assert abs(m[14] - Pi[1, 2]) < tol
        assert abs(m[15] - Pi[0, 2]) < tol


def test_d3q19_third_moment_rows(orc):
    """q rows follow from the third moment, the corrected (A7):
    sum e_i e_j e_k g_eq = c_s^2 sigma (u_k d_ij + u_i d_jk + u_j d_ik).
    q_x = sum (5 e^2 - 9) e_x g_eq = 5 sum e^2 e_x g_eq - 9 sigma u_x.
    The m rows (odd, cubic, traceless combinations) vanish at equilibrium.
    """
    t = orc.tables()
    M, e = t["M"], t["e"].astype(float)
    rng = np.random.default_rng(7)
    cs2 = 1.0 / 3.0
    for _ in range(30):
        eps, P, u, sigma = _rand_state(rng)
        g = orc.geq(eps, P, u)
        m = M @ g
        third = cs2 * sigma * 5.0 * u  # sum_j (u_i d_jj + 2 u_j d_ij) = 5 u_i
        for row, i in ((4, 0), (6, 1), (8, 2)):
            assert abs(m[row] - (5 * third[i] - 9 * sigma * u[i])) < 1e-13 * sigma
        assert np.abs(m[16:19]).max() < 1e-13 * sigma
