"""Oracle pins: what the paper's analysis fixes for whole runs.

* Stationarity of a uniform state (any u), periodic and zero-gradient.
* Conservation of the lattice sums of n gamma, T^00 = sigma - P and
  T^0i = sigma u_i under periodic boundaries (Eqs. 2-3).
* Shear-wave decay with the viscosity set by tau_v:
  eta = (tau_v - dt/2) c_s^2 sigma / gamma (text after Eq. 10 and after Eq. 36),
  so a small shear wave decays at nu k^2 with nu = (tau_v - 1/2)/3.
* Particle-number diffusion of Eq. (23): at u = 0 and uniform P the
  particle number obeys a diffusion equation with phi = c_s^2 (tau_f - dt/2).
* Bulk relaxation trend: a sound wave is damped more when tau_e grows (the
  bulk viscosity after Eq. 36 grows with tau_e - dt/2).
* Sound attenuation, quantitatively: at rest with P = eps/3 (chi = 0), a
  small plane sound wave along y obeys the linearised Eqs. (24)-(25) with
  Pi_yy = ((2 - 2/D) eta + varsigma) d_y u, which gives omega = +-k c_s - i G,
  G = ((2 - 2/D) eta + varsigma) k^2 / (2 (eps + P)). D2Q9 (Eq. 36, D = 2):
  eta = (tau_v - 1/2) c_s^2 sigma, varsigma = (tau_e - 1/2) c_s^2 sigma, so
  G = k^2 (tau_v + tau_e - 1) / 6. D3Q19 (D = 3): the same expansion of the
  moment basis gives varsigma = (2/3)(tau_e - 1/2) c_s^2 sigma, so
  G = k^2 ((4/3)(tau_v - 1/2) + (2/3)(tau_e - 1/2)) / 6. The frequency is
  k c_s with c_s^2 = 1/3.
"""

import numpy as np
import pytest

import workloads as wl


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1), (0, 1, 0)])
def test_uniform_state_is_stationary(orc, bc):
    prob = wl.uniform(5, 4, 6, n=1.3, eps=2.1, u=(0.3, -0.2, 0.1), bc=bc,
                      tau_f=0.7, tau_v=0.9, tau_e=0.6, tau_eps=1.1)
    st = orc.State.init(prob)
    f0, g0 = st.f.copy(), st.g.copy()
    st.step(20)
    assert np.abs(st.f - f0).max() < 1e-14 * np.abs(f0).max()
    assert np.abs(st.g - g0).max() < 1e-14 * np.abs(g0).max()
    F = st.fields()
    assert np.abs(F["u"][0] - 0.3).max() < 1e-14
    assert np.abs(F["n"] - 1.3).max() < 1e-14
    assert np.abs(F["eps"] - 2.1).max() < 1e-13


def test_periodic_conservation(orc):
    prob = wl.random_modes(12, 10, 14, seed=5, umax=0.2, amp=0.1)
    st = orc.State.init(prob)
    s0 = st.fields()["sums"]
    st.step(60)
    s1 = st.fields()["sums"]
    scale = np.abs(s0[:2]).max()
    assert np.abs(s1 - s0).max() < 1e-13 * scale
    assert st.bad == 0


def _amplitude(field, k, axis_len):
    y = np.arange(axis_len)
    return 2.0 / axis_len * (field * np.sin(k * y)).sum()


@pytest.mark.parametrize("tau_v,tau_e,tau_eps", [(0.8, 0.55, 0.7), (1.1, 1.1, 1.1),
                                                 (0.6, 0.9, 0.6)])
def test_shear_wave_decay(orc, tau_v, tau_e, tau_eps):
    L = 128
    k = 2 * np.pi / L
    U = 1e-3
    prob = wl.uniform(1, L, 1, n=1.0, eps=1.0, tau_f=0.8, tau_v=tau_v, tau_e=tau_e,
                      tau_eps=tau_eps)
    prob.u[0, 0, :, 0] = U * np.sin(k * np.arange(L))
    st = orc.State.init(prob)
    t0, t1 = 200, 1800
    st.step(t0)
    a0 = _amplitude(st.fields()["u"][0, 0, :, 0], k, L)
    st.step(t1 - t0)
    a1 = _amplitude(st.fields()["u"][0, 0, :, 0], k, L)
    rate = -np.log(a1 / a0) / (t1 - t0)
    nu = (tau_v - 0.5) / 3.0
    assert abs(rate / (nu * k * k) - 1.0) < 0.01


@pytest.mark.parametrize("tau_f", [0.6, 0.9, 1.4])
def test_particle_number_diffusion(orc, tau_f):
    L = 64
    k = 2 * np.pi / L
    prob = wl.uniform(1, 1, L, n=1.0, eps=1.0, tau_f=tau_f, tau_v=0.8, tau_e=0.55,
                      tau_eps=0.7)
    z = np.arange(L)
    prob.n[:, 0, 0] = 1.0 + 1e-3 * np.sin(k * z)
    st = orc.State.init(prob)
    t0, t1 = 50, 450
    st.step(t0)
    a0 = _amplitude(st.fields()["n"][:, 0, 0] - 1.0, k, L)
    st.step(t1 - t0)
    a1 = _amplitude(st.fields()["n"][:, 0, 0] - 1.0, k, L)
    rate = -np.log(a1 / a0) / (t1 - t0)
    phi = (tau_f - 0.5) / 3.0
    assert abs(rate / (phi * k * k) - 1.0) < 0.01
    # g never reads f: the flow stays at rest (to rounding of M^-1)
    assert np.abs(st.fields()["u"]).max() < 1e-13


def test_particle_number_depends_on_tau_f_only_through_f(orc):
    """Eq. (23): the shock-tube particle number depends on tau_f while the
    energy-momentum fields do not (g never reads f)."""
    outs = {}
    for tf in (0.55, 0.9):
        prob = wl.shock_tube(200, tau=0.9, tau_f=tf)
        st = orc.run(prob, 100)
        outs[tf] = st.fields()
    a, b = outs[0.55], outs[0.9]
    assert np.array_equal(a["eps"], b["eps"]) and np.array_equal(a["u"], b["u"])
    assert np.abs(a["n"] - b["n"]).max() > 1e-3
    # larger tau_f -> more diffusion -> smoother (smaller total variation)
    tv = lambda x: np.abs(np.diff(x.ravel())).sum()
    assert tv(b["n"]) < tv(a["n"])


def test_bulk_relaxation_damps_sound(orc):
    L = 64
    k = 2 * np.pi / L
    amps = []
    for tau_e in (0.52, 0.8, 1.2):
        prob = wl.uniform(1, 1, L, n=1.0, eps=1.0, tau_f=0.8, tau_v=0.8, tau_e=tau_e,
                          tau_eps=0.8)
        prob.eps[:, 0, 0] = 1.0 + 1e-3 * np.sin(k * np.arange(L))
        st = orc.State.init(prob)
        st.step(300)
        F = st.fields()
        # acoustic energy: pressure and momentum fluctuations
        amps.append(np.abs(F["eps"] - F["eps"].mean()).max() + np.abs(F["u"][2]).max())
    assert amps[0] > amps[1] > amps[2]


@pytest.mark.parametrize("lattice,tau_v,tau_e", [("d2q9", 0.8, 0.55), ("d2q9", 0.6, 1.0),
                                                  ("d3q19", 0.8, 0.55), ("d3q19", 1.2, 0.7)])
def test_sound_attenuation_matches_the_bulk_and_shear_viscosities(orc, lattice, tau_v, tau_e):
    from scipy.optimize import curve_fit
    L, T, amp = 128, 1200, 1e-4
    k = 2 * np.pi / L
    prob = wl.uniform(1, L, 1, n=1.0, eps=1.0, tau_f=0.8, tau_v=tau_v, tau_e=tau_e,
                      tau_eps=0.9)
    prob.params.lattice = lattice
    y = np.arange(L)
    prob.eps[0, :, 0] = 1.0 + amp * np.cos(k * y)
    st = orc.State.init(prob)
    a = np.empty(T)
    for t in range(T):
        st.step(1)
        a[t] = 2.0 / L * ((st.fields()["eps"][0, :, 0] - 1.0) * np.cos(k * y)).sum()
    t = np.arange(1, T + 1)
    (A, G, w, p), _ = curve_fit(lambda t, A, G, w, p: A * np.exp(-G * t) * np.cos(w * t + p), t,
                                a, p0=[amp, 1e-4, k / np.sqrt(3.0), 0.0], maxfev=20000)
    if lattice == "d2q9":
        want = k * k / 6.0 * (tau_v + tau_e - 1.0)
    else:
        want = k * k / 6.0 * (4.0 / 3.0 * (tau_v - 0.5) + 2.0 / 3.0 * (tau_e - 0.5))
    assert abs(G / want - 1.0) < 2e-3, (G, want)
    assert abs(w / (k / np.sqrt(3.0)) - 1.0) < 1e-3


def test_particle_bump_is_carried_by_the_flow(orc):
    """Eq. (23) convection: a particle-number bump in a uniform flow u_z moves
    downstream at u_z (pins the direction of streaming, Eqs. 5-6)."""
    L = 128
    uz = 0.1
    prob = wl.uniform(1, 1, L, n=1.0, eps=1.0, u=(0.0, 0.0, uz), tau_f=0.52, tau_v=0.8,
                      tau_e=0.8, tau_eps=0.8)
    z = np.arange(L)
    prob.n[:, 0, 0] = 1.0 + 1e-3 * np.exp(-((z - 40.0) / 4.0) ** 2)
    st = orc.State.init(prob)

    def centroid():
        d = st.fields()["n"][:, 0, 0] - 1.0
        return (d * z).sum() / d.sum()

    c0 = centroid()
    st.step(200)
    assert abs((centroid() - c0) - uz * 200) < 0.5


def test_open_ends_keep_far_field(orc):
    """Zero-gradient ("open") ends leave a uniform end region untouched until
    the shock waves arrive; a periodic tube instead starts a second Riemann
    problem where the two ends meet."""
    L = 200
    res = {}
    for bc in (1, 0):
        prob = wl.shock_tube(L, tau=0.9)
        prob.params.bc = (0, 0, bc)
        st = orc.run(prob, 40)
        res[bc] = st.fields()["eps"][:, 0, 0]
    eps0 = wl.shock_tube(L)
    assert np.abs(res[1][:20] - eps0.eps[:20, 0, 0]).max() < 1e-12
    assert np.abs(res[1][-20:] - eps0.eps[-20:, 0, 0]).max() < 1e-12
    assert np.abs(res[0][:20] - eps0.eps[:20, 0, 0]).max() > 1e-3


# Non-hydrodynamic modes of g over whole runs: on a uniform periodic lattice
# streaming maps every population onto an equal one, and the conserved sums
# (hence the equilibria) do not change, so a perturbation along one moment row
# decays by (1 - 1/tau) per step, tau the rate Eq. (31) gives that row. The
# rows are written here from their closed forms in |e|^2 (the bulk row
# e = 19 r^2 - 30 (D3Q19), 3 r^2 - 4 (D2Q9) with tau_e; the energy-square row
# (21 r^4 - 53 r^2 + 24)/2, (9 r^4 - 21 r^2 + 8)/2 with tau_eps), not taken
# from the oracle's basis, so a wrong row, norm or rate mapping breaks the
# single-exponential decay.
_ROWS = {
    ("d3q19", "e"): (lambda r2: 19.0 * r2 - 30.0, "tau_e"),
    ("d3q19", "eps"): (lambda r2: (21.0 * r2 * r2 - 53.0 * r2 + 24.0) / 2.0, "tau_eps"),
    ("d2q9", "e"): (lambda r2: 3.0 * r2 - 4.0, "tau_e"),
    ("d2q9", "eps"): (lambda r2: (9.0 * r2 * r2 - 21.0 * r2 + 8.0) / 2.0, "tau_eps"),
}


@pytest.mark.parametrize("lattice,row", list(_ROWS), ids=lambda v: str(v))
def test_ghost_mode_decays_at_its_rate(lattice, row):
    import oracle
    taus = dict(tau_f=0.7, tau_v=0.8, tau_e=0.6, tau_eps=1.3, tau_q=1.1)
    if lattice == "d2q9":
        prob = wl.uniform(4, 5, 1, n=1.0, eps=1.0, u=(0.12, -0.07, 0.0), **taus)
        prob.params.lattice = "d2q9"
        e = oracle.d2q9_tables()["e"]
    else:
        prob = wl.uniform(4, 5, 3, n=1.0, eps=1.0, u=(0.12, -0.07, 0.05), **taus)
        e = oracle.tables()["e"]
    poly, rate = _ROWS[(lattice, row)]
    r2 = (np.asarray(e, dtype=float) ** 2).sum(axis=1)
    phi = poly(r2)
    delta = 1e-3
    base = oracle.State.init(prob)
    pert = oracle.State.init(prob)
    pert.g += (delta * phi / (phi * phi).sum())[:, None, None, None]
    T = 12
    base.step(T)
    pert.step(T)
    m = np.tensordot(phi, pert.g - base.g, axes=1)  # the row's moment in every cell
    expect = delta * (1.0 - 1.0 / taus[rate]) ** T
    assert np.abs(m - expect).max() < 1e-9 * abs(delta)
    # the perturbation stays in that row: the other moments of the difference
    # (here the plain sum and the other ghost row) stay at rounding level
    assert np.abs((pert.g - base.g).sum(axis=0)).max() < 1e-10 * delta
    other = [k for k in _ROWS if k[0] == lattice and k[1] != row][0]
    phi2 = _ROWS[other][0](r2)
    assert np.abs(np.tensordot(phi2, pert.g - base.g, axes=1)).max() < 1e-10 * delta
