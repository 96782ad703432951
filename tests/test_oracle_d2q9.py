"""Oracle pins for the D2Q9 MRT model of Sec. V.A (Eqs. 30-35) and its runs.

Each pin is checked against something other than the oracle itself:

* Lattice: D2Q9 weights are isotropic to fourth order with c_s^2 = 1/3; the
  basis rows are orthogonal with the squared norms of the polynomials; the
  conserved rows are the Eq. (10) moments. (The printed Eq. (34) is pinned
  in test_oracle_lattice.py against tests/golden/eq34_d2q9_meq.txt.)
* Equilibria: f_eq and g_eq (Eqs. 7, 32-33) carry the moments the
  constraints fix: n gamma, n gamma u, sigma - P, sigma u, P delta + sigma u u.
  At rest g_eq = (4P/3, P/3, P/12).
* Collision: with every rate 1/tau the MRT of Eq. (35) is the BGK of Eq. (6);
  each non-conserved moment relaxes with its own rate of Eq. (31); N, E, M
  are conserved per cell.
* Whole runs: a uniform state is stationary (periodic and zero-gradient);
  sums are conserved on periodic lattices; a shear wave decays at
  nu = (tau_v - 1/2)/3; particle number diffuses at c_s^2 (tau_f - 1/2);
  sound damping grows with tau_e.
* Sec. V.B: on the 4 x 800 shock tube at t = 400 the Cases A and B (tau_e =
  tau_v) show a velocity jump at the membrane, which reducing tau_e (Cases C
  and D) removes, and tau_q has no visible effect (A versus B).
"""

import numpy as np
import pytest

import workloads as wl


def _d2(prob):
    prob.params.lattice = "d2q9"
    return prob


def test_weights_isotropy(orc):
    t = orc.d2q9_tables()
    e = t["e"].astype(float)
    w = t["w"]
    assert abs(w.sum() - 1.0) < 1e-15
    d = np.eye(2)
    second = np.einsum("a,ai,aj->ij", w, e, e)
    assert np.abs(second - d / 3.0).max() < 1e-15
    fourth = np.einsum("a,ai,aj,ak,al->ijkl", w, e, e, e, e)
    iso = (np.einsum("ij,kl->ijkl", d, d) + np.einsum("ik,jl->ijkl", d, d) +
           np.einsum("il,jk->ijkl", d, d)) / 9.0
    assert np.abs(fourth - iso).max() < 1e-15
    # odd moments vanish
    assert np.abs(np.einsum("a,ai->i", w, e)).max() < 1e-16
    # opposite directions come in pairs
    for a in range(9):
        assert any((e[b] == -e[a]).all() for b in range(9))


def test_basis_norms_and_conserved_rows(orc):
    t = orc.d2q9_tables()
    M = t["M"]
    e = t["e"]
    G = M @ M.T
    assert np.abs(G - np.diag(np.diag(G))).max() == 0.0
    assert np.array_equal(np.diag(G), [9, 36, 36, 6, 12, 6, 12, 4, 4])
    assert np.linalg.matrix_rank(M) == 9
    assert np.array_equal(M[0], np.ones(9))
    assert np.array_equal(M[3], e[:, 0]) and np.array_equal(M[5], e[:, 1])


@pytest.mark.parametrize("seed", range(6))
def test_equilibrium_moments(orc, seed):
    rng = np.random.default_rng(seed)
    t = orc.d2q9_tables()
    e = t["e"].astype(float)
    u = rng.uniform(-0.3, 0.3, 2)
    eps = rng.uniform(0.5, 2.0)
    n = rng.uniform(0.5, 2.0)
    P = eps / 3.0
    gam = 1.0 / np.sqrt(1.0 - u @ u)
    sigma = (eps + P) * gam ** 2
    g = orc.d2q9_geq(sigma, P, u)
    assert abs(g.sum() - (sigma - P)) < 1e-14 * sigma
    assert np.abs(e.T @ g - sigma * u).max() < 1e-14 * sigma
    second = np.einsum("a,ai,aj->ij", g, e, e)
    assert np.abs(second - (P * np.eye(2) + sigma * np.outer(u, u))).max() < 1e-14 * sigma
    f = orc.d2q9_feq(n, gam, u)
    assert abs(f.sum() - n * gam) < 1e-14 * n
    assert np.abs(e.T @ f - n * gam * u).max() < 1e-14 * n


def test_rest_state_values(orc):
    P = 0.37
    g = orc.d2q9_geq(4.0 * P, P, np.zeros(2))
    w = orc.d2q9_tables()["w"]
    want = np.where(w == 4.0 / 9.0, 4.0 * P / 3.0, np.where(w == 1.0 / 9.0, P / 3.0, P / 12.0))
    assert np.abs(g - want).max() < 1e-15 * P


def _cell_state(orc, rng, amp=0.05):
    u = rng.uniform(-0.25, 0.25, 2)
    eps = rng.uniform(0.8, 1.5)
    n = rng.uniform(0.8, 1.5)
    P = eps / 3.0
    gam = 1.0 / np.sqrt(1.0 - u @ u)
    g = orc.d2q9_geq((eps + P) * gam ** 2, P, u)
    f = orc.d2q9_feq(n, gam, u)
    g = g * (1.0 + amp * rng.standard_normal(9))
    f = f * (1.0 + amp * rng.standard_normal(9))
    return f, g


def _params(**kw):
    p = wl.Params(1, 1, 1, **kw)
    p.lattice = "d2q9"
    return p


def _fields_of(orc, f, g):
    e = orc.d2q9_tables()["e"].astype(float)
    M = np.array([*(e.T @ g), 0.0])
    ok, F = orc.recover(f.sum(), g.sum(), M)
    return ok, F


@pytest.mark.parametrize("seed", range(5))
def test_mrt_equals_bgk_when_rates_equal(orc, seed):
    rng = np.random.default_rng(100 + seed)
    f, g = _cell_state(orc, rng)
    tau = rng.uniform(0.55, 3.0)
    p = _params(tau_f=0.7, tau_v=tau, tau_e=tau, tau_eps=tau, tau_q=tau)
    ok, fo, go = orc.collide_cell(p, f, g)
    assert ok
    ok, F = _fields_of(orc, f, g)
    u = np.array([F["ux"], F["uy"]])
    geq = orc.d2q9_geq(F["sigma"], F["P"], u)
    assert np.abs(go - (g - (g - geq) / tau)).max() < 1e-14 * np.abs(g).max()
    feq = orc.d2q9_feq(F["n"], F["gamma"], u)
    assert np.abs(fo - (f - (f - feq) / 0.7)).max() < 1e-14 * np.abs(f).max()


@pytest.mark.parametrize("row,name", [(1, "tau_e"), (2, "tau_eps"), (4, "tau_q"), (6, "tau_q"),
                                      (7, "tau_v"), (8, "tau_v")])
def test_each_moment_relaxes_with_its_own_rate(orc, row, name):
    rng = np.random.default_rng(7 + row)
    f, g = _cell_state(orc, rng)
    taus = dict(tau_f=0.9, tau_v=0.8, tau_e=0.63, tau_eps=1.7, tau_q=1.21)
    p = _params(**taus)
    ok, fo, go = orc.collide_cell(p, f, g)
    ok, F = _fields_of(orc, f, g)
    M = orc.d2q9_tables()["M"]
    meq = M @ orc.d2q9_geq(F["sigma"], F["P"], np.array([F["ux"], F["uy"]]))
    m, ms = M @ g, M @ go
    s = 1.0 / taus[name]
    assert abs((ms[row] - meq[row]) - (1.0 - s) * (m[row] - meq[row])) < 1e-13 * np.abs(m).max()
    for k in (0, 3, 5):  # conserved rows
        assert abs(ms[k] - m[k]) < 1e-14 * np.abs(m).max()


def test_inadmissible_cell_is_left_alone(orc):
    p = _params(tau_f=0.9, tau_v=0.9, tau_e=0.9, tau_eps=0.9)
    f = np.full(9, 0.1)
    g = np.zeros(9)
    g[1] = 1.0  # |M| = E: no subluminal state
    ok, fo, go = orc.collide_cell(p, f, g)
    assert not ok and np.array_equal(fo, f) and np.array_equal(go, g)


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 0), (0, 1, 0)])
def test_uniform_state_is_stationary(orc, bc):
    prob = _d2(wl.uniform(5, 7, 1, n=1.3, eps=2.1, u=(0.3, -0.2, 0.0), bc=bc, tau_f=0.7,
                          tau_v=0.9, tau_e=0.6, tau_eps=1.1, tau_q=1.3))
    st = orc.State.init(prob)
    f0, g0 = st.f.copy(), st.g.copy()
    st.step(20)
    assert np.abs(st.f - f0).max() < 1e-14 * np.abs(f0).max()
    assert np.abs(st.g - g0).max() < 1e-14 * np.abs(g0).max()
    F = st.fields()
    assert np.abs(F["u"][0] - 0.3).max() < 1e-14 and np.abs(F["u"][2]).max() == 0.0


def test_periodic_conservation(orc):
    prob = _d2(wl.random_modes(24, 18, 1, seed=5, umax=0.2, amp=0.1))
    st = orc.State.init(prob)
    s0 = st.fields()["sums"]
    st.step(80)
    s1 = st.fields()["sums"]
    assert np.abs(s1 - s0).max() < 1e-13 * np.abs(s0[:2]).max()
    assert st.bad == 0 and s1[4] == 0.0


def _amplitude(field, k, n):
    y = np.arange(n)
    return 2.0 / n * (field * np.sin(k * y)).sum()


@pytest.mark.parametrize("tau_v,tau_e,tau_q", [(0.8, 0.55, 0.8), (1.1, 0.7, 1.5)])
def test_shear_wave_decay(orc, tau_v, tau_e, tau_q):
    L = 128
    k = 2 * np.pi / L
    prob = _d2(wl.uniform(1, L, 1, tau_f=0.8, tau_v=tau_v, tau_e=tau_e, tau_eps=0.7,
                          tau_q=tau_q))
    prob.u[0, 0, :, 0] = 1e-3 * np.sin(k * np.arange(L))
    st = orc.State.init(prob)
    st.step(200)
    a0 = _amplitude(st.fields()["u"][0, 0, :, 0], k, L)
    st.step(1600)
    a1 = _amplitude(st.fields()["u"][0, 0, :, 0], k, L)
    rate = -np.log(a1 / a0) / 1600
    assert abs(rate / ((tau_v - 0.5) / 3.0 * k * k) - 1.0) < 0.01


@pytest.mark.parametrize("tau_f", [0.6, 1.2])
def test_particle_number_diffusion(orc, tau_f):
    L = 64
    k = 2 * np.pi / L
    prob = _d2(wl.uniform(L, 1, 1, tau_f=tau_f, tau_v=0.8, tau_e=0.55, tau_eps=0.7))
    prob.n[0, 0, :] = 1.0 + 1e-3 * np.sin(k * np.arange(L))
    st = orc.State.init(prob)
    st.step(50)
    a0 = _amplitude(st.fields()["n"][0, 0, :] - 1.0, k, L)
    st.step(400)
    a1 = _amplitude(st.fields()["n"][0, 0, :] - 1.0, k, L)
    rate = -np.log(a1 / a0) / 400
    assert abs(rate / ((tau_f - 0.5) / 3.0 * k * k) - 1.0) < 0.01


def test_bulk_relaxation_damps_sound(orc):
    L = 64
    k = 2 * np.pi / L
    amps = []
    for tau_e in (0.52, 0.8, 1.2):
        prob = _d2(wl.uniform(1, L, 1, tau_f=0.8, tau_v=0.8, tau_e=tau_e, tau_eps=0.8))
        prob.eps[0, :, 0] = 1.0 + 1e-3 * np.sin(k * np.arange(L))
        st = orc.State.init(prob)
        st.step(300)
        F = st.fields()
        amps.append(np.abs(F["eps"] - F["eps"].mean()).max() + np.abs(F["u"][1]).max())
    assert amps[0] > amps[1] > amps[2]


def test_sec5_cases_membrane_jump(orc):
    """Sec. V.B, 4 x 800 tube at t = 400 (a = 1/20): a velocity jump at the
    membrane with tau_e = tau_v (Cases A, B), none once tau_e is reduced
    (Cases C, D); tau_q leaves the profile unchanged to within 1e-4."""
    out = {}
    for case in "ABCD":
        F = orc.run(wl.qgp_tube_2d(case), 400).fields()
        uz = F["u"][1, 0, :, 0]
        assert np.ptp(F["u"][1, 0], axis=1).max() == 0.0  # uniform across the periodic x
        assert F["bad"] == 0
        out[case] = uz
    jump = {c: abs(out[c][400] - out[c][399]) for c in "ABCD"}
    assert jump["A"] > 0.01 and jump["B"] > 0.01
    assert jump["C"] < 0.1 * jump["A"] and jump["D"] < 0.1 * jump["A"]
    assert np.abs(out["A"] - out["B"]).max() < 1e-4 * np.abs(out["A"]).max()
    # weakly relativistic: beta around 0.2
    assert 0.15 < out["D"].max() < 0.25


@pytest.mark.parametrize("lattice,dims,bc,axis", [("d2q9", (12, 9, 1), (0, 1, 0), 3),
                                                  ("d2q9", (12, 9, 1), (1, 0, 0), 2),
                                                  ("d3q19", (6, 7, 5), (0, 1, 1), 3),
                                                  ("d3q19", (6, 7, 5), (1, 0, 1), 2),
                                                  ("d3q19", (6, 7, 5), (1, 1, 0), 1)])
def test_periodic_axis_is_translation_invariant(orc, lattice, dims, bc, axis):
    """Along a periodic axis the update commutes with a cyclic shift of the
    fields, whatever the other axes do. ``axis`` is the population axis
    (1 = z, 2 = y, 3 = x); fields have one axis less."""
    prob = wl.random_modes(*dims, seed=21, umax=0.25, amp=0.1, bc=bc)
    prob.params.lattice = lattice
    shifted = wl.random_modes(*dims, seed=21, umax=0.25, amp=0.1, bc=bc)
    shifted.params.lattice = lattice
    shifted.n = np.roll(prob.n, 3, axis=axis - 1)
    shifted.eps = np.roll(prob.eps, 3, axis=axis - 1)
    shifted.u = np.roll(prob.u, 3, axis=axis)
    a = orc.run(prob, 12)
    b = orc.run(shifted, 12)
    assert np.abs(np.roll(a.g, 3, axis=axis) - b.g).max() < 1e-14 * np.abs(a.g).max()
    assert np.abs(np.roll(a.f, 3, axis=axis) - b.f).max() < 1e-14 * np.abs(a.f).max()
