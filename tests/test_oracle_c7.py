"""Oracle pins for the correction term of Eqs. (37)-(38) on the D2Q9 model.

The correction adds (I - S/2) C with C = (0, ..., C_7, 0) to the collision,
C_7 built from y-derivatives (the flow axis) of the recovered fields. Pins:

* Chapman-Enskog: for a flow along y with uniform u and a density gradient,
  the first-order flux of row 7 carries an error proportional to u d(sigma)
  that the correction exists to cancel. The coefficient is derived here with
  sympy from the D2Q9 equilibria (Eqs. 32-33), independently of Eq. (38),
  and the change of m_7 that the oracle's correction makes in one step must
  equal (1 - s_v/2) times it (sign and size).
* It vanishes where its derivatives vanish: a uniform state stays uniform,
  and a flow that does not vary along y gives the uncorrected run bit for bit.
* Homogeneity: every term is of degree one in (sigma, P), so scaling eps and
  n by 4 scales the corrected populations by 4 exactly.
* Mirror symmetry about the tube centre (y -> -y, u_y -> -u_y) is kept.
* Every term at every order in u, the gamma term and theta included: sympy
  carries the row-7 residual along the route Sec. V.B names (the change of
  Eq. 28, gamma du -> d(gamma u), the velocity terms of d_t1(sigma u^2)),
  which gives the printed Eq. (38) exactly; the correction the oracle applies
  on smooth tubes at |u| up to 0.55 equals that expansion up to the O(k^2)
  gap of central differences.
"""

import numpy as np
import pytest

import workloads as wl


def _tube(L=64, nx=1, bc=(0, 0, 0), correction=1, **tau):
    t = dict(tau_f=0.7, tau_v=1.3, tau_e=0.8, tau_eps=0.9, tau_q=1.1)
    t.update(tau)
    prob = wl.uniform(nx, L, 1, bc=bc, **t)
    prob.params.lattice = "d2q9"
    prob.params.correction = correction
    return prob


def _ce_row7_dsigma_coefficient(u0):
    """Coefficient of d(sigma)/dy in the first-order row-7 term
    d_t1 m7_eq + d_y F7 of the D2Q9 model, for a 1D flow along y, from a
    Chapman-Enskog expansion of the equilibria of Eqs. (32)-(33)."""
    sp = pytest.importorskip("sympy")
    y = sp.symbols("y")
    s = sp.Function("sigma")(y)
    u = sp.Function("u")(y)
    P = s * (1 - u ** 2) / 4  # P = eps/3, sigma = (eps + P) gamma^2
    c2 = sp.Rational(1, 3)
    E = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
    W = [sp.Rational(4, 9)] + [sp.Rational(1, 9)] * 4 + [sp.Rational(1, 36)] * 4

    def geq(a):
        eu = E[a][1] * u
        if a == 0:
            return W[0] * s * (sp.Rational(9, 4) - P * (5 + 9 * c2) / (4 * s * c2)
                               - u ** 2 / (2 * c2))
        return W[a] * s * (P / (s * c2) + eu / c2 + eu ** 2 / (2 * c2 ** 2) - u ** 2 / (2 * c2))

    g = [geq(a) for a in range(9)]
    r7 = [ex * ex - ey * ey for ex, ey in E]
    m7 = sum(r * q for r, q in zip(r7, g))
    F7 = sum(r * E[a][1] * g[a] for a, r in enumerate(r7))
    En = sum(g)
    Mo = sum(E[a][1] * g[a] for a in range(9))
    Pyy = sum(E[a][1] ** 2 * g[a] for a in range(9))
    S, U = sp.symbols("S U")
    J = sp.Matrix([[sp.diff(En.subs({s: S, u: U}), v) for v in (S, U)],
                   [sp.diff(Mo.subs({s: S, u: U}), v) for v in (S, U)]])
    rates = J.inv() * sp.Matrix([-sp.diff(Mo, y), -sp.diff(Pyy, y)]).subs({s: S, u: U})
    m7f = m7.subs({s: S, u: U})
    dt_m7 = (sp.diff(m7f, S) * rates[0] + sp.diff(m7f, U) * rates[1]).subs({S: s, U: u})
    D7 = dt_m7 + sp.diff(F7, y)
    ds, du = sp.symbols("ds du")
    D7 = D7.subs({sp.Derivative(s, y): ds, sp.Derivative(u, y): du})
    coef = sp.diff(sp.expand(D7), ds).subs({du: 0})
    return float(coef.subs({u: u0}))


def test_correction_cancels_the_leading_chapman_enskog_error(orc):
    # small u: the printed term and the expansion differ at O(u^3) (relative
    # 9 u^2, 0.4 % here), the leading O(u) part must match
    L, u0, amp = 256, 0.02, 0.01
    k = 2 * np.pi / L
    y = np.arange(L)
    runs = {}
    for corr in (0, 1):
        prob = _tube(L, correction=corr, tau_v=1.7)
        prob.eps[0, :, 0] = 1.0 + amp * np.sin(k * y)
        prob.u[1] = u0
        st = orc.run(prob, 1)
        runs[corr] = st.g.reshape(9, L)
    M = orc.d2q9_tables()["M"]
    dm7 = (M @ (runs[1] - runs[0]))[7]
    # sigma = 4 eps gamma^2 / 3 at uniform u; d(sigma)/dy of the initial field
    gam2 = 1.0 / (1.0 - u0 * u0)
    dsig = 4.0 / 3.0 * gam2 * amp * k * np.cos(k * y)
    want = (1.0 - 0.5 / 1.7) * _ce_row7_dsigma_coefficient(u0) * dsig
    fit = (dm7 @ want) / (want @ want)
    assert abs(fit - 1.0) < 0.01, fit
    assert np.abs(dm7 - want).max() < 0.02 * np.abs(want).max()


@pytest.mark.parametrize("bc", [(0, 0, 0), (0, 1, 0)])
def test_uniform_state_stays_uniform(orc, bc):
    prob = _tube(40, nx=3, bc=bc)
    prob.eps[:] = 1.7
    prob.u[1] = 0.3
    prob.u[0] = -0.1
    st = orc.State.init(prob)
    f0, g0 = st.f.copy(), st.g.copy()
    st.step(15)
    assert np.abs(st.g - g0).max() < 1e-14 * np.abs(g0).max()
    assert np.abs(st.f - f0).max() < 1e-14 * np.abs(f0).max()


def test_no_effect_without_y_variation(orc):
    """Fields that vary along x only: every y-derivative is zero, so the
    corrected and uncorrected runs are identical bit for bit."""
    out = []
    for corr in (0, 1):
        prob = _tube(6, nx=48, bc=(0, 1, 0), correction=corr)
        x = np.arange(48)
        prob.eps[0] = 1.0 + 0.2 * np.sin(2 * np.pi * x / 48)[None, :]
        prob.u[1, 0] = 0.2 * np.cos(2 * np.pi * x / 48)[None, :]
        out.append(orc.run(prob, 20).g)
    assert np.array_equal(out[0], out[1])


def test_correction_changes_a_flow_along_y(orc):
    out = []
    for corr in (0, 1):
        prob = _tube(64, correction=corr)
        prob.eps[0, :, 0] = 1.0 + 0.3 * np.sin(2 * np.pi * np.arange(64) / 64)
        prob.u[1] = 0.2
        out.append(orc.run(prob, 20).g)
    assert np.abs(out[0] - out[1]).max() > 1e-6 * np.abs(out[0]).max()


def test_homogeneous_of_degree_one(orc):
    base = wl.qgp_tube_2d("D", moderate=True, a=1.0 / 30.0, correction=True, length=200)
    scaled = wl.qgp_tube_2d("D", moderate=True, a=1.0 / 30.0, correction=True, length=200)
    scaled.eps = 4.0 * base.eps
    scaled.n = 4.0 * base.n
    a = orc.run(base, 60)
    b = orc.run(scaled, 60)
    assert np.array_equal(4.0 * a.g, b.g) and np.array_equal(4.0 * a.f, b.f)


def test_mirror_symmetry(orc):
    L = 120
    yc = (L - 1) / 2.0
    y = np.arange(L) - yc
    prob = _tube(L, nx=2, bc=(0, 1, 0), tau_v=3.0, tau_e=0.9, tau_eps=0.9, tau_q=3.0)
    prob.eps[0] = (1.0 + 0.5 * np.exp(-(y / 12.0) ** 2))[:, None]
    prob.u[1, 0] = (0.3 * np.tanh(y / 10.0))[:, None]
    st = orc.run(prob, 50)
    F = st.fields()
    eps, uy = F["eps"][0, :, 0], F["u"][1, 0, :, 0]
    assert np.abs(eps - eps[::-1]).max() < 1e-12 * eps.max()
    assert np.abs(uy + uy[::-1]).max() < 1e-12


def test_dependence_cone_is_two_cells_a_step(orc):
    """A corrected step reads the y-neighbours' fields after their pull, so
    after K steps a cell depends on cells up to 2K away along y: a window of
    half-width 2K reproduces the full run exactly, one of half-width K does
    not (the full-size GPU tests rely on the former)."""
    prob = wl.random_modes(48, 40, 1, seed=7, umax=0.1, amp=0.05, tau_v=0.8, tau_e=0.55,
                           tau_eps=0.7, tau_f=0.8)
    prob.params.lattice = "d2q9"
    prob.params.correction = 1
    K = 3
    full = orc.run(prob, K)
    for radius, exact in ((2, True), (1, False)):
        d = 0.0
        for c in ((0, 5, 7), (0, 20, 30), (0, 39, 0)):
            sub, loc = wl.window(prob, c, radius * K)
            st = orc.run(sub, K)
            d = max(d, np.abs(st.g[(slice(None),) + loc] - full.g[(slice(None),) + c]).max())
        assert (d == 0.0) == exact, (radius, d)


def _c7_from_the_expansion():
    """C_7 of this basis' row 7 (e_x^2 - e_y^2, flow along y) derived along the
    route Sec. V.B describes, as a function of (sigma, u, d sigma/dy, du/dy).

    The first-order Chapman-Enskog residual of row 7 is
    D_7 = d_t1 m7_eq + d_y F_7, with m7_eq, F_7 and the Euler equations of
    the model (d_t1 (sigma - P) = -d_y (sigma u), d_t1 (sigma u) =
    -d_y (sigma u^2 + P)) all taken from the moments of the D2Q9 equilibria
    (Eqs. 32-33). The correction replaces D_7 by the residual that gives the
    shear stress eta d(gamma u) of Eq. (36) with no other term: the
    isotropic-equilibrium residual -2 c_s^2 sigma gamma^-1 d(gamma u), i.e.
    the shear term of Eq. (36) with gamma du changed to d(gamma u). Two
    readings complete the paper's account of the velocity terms from
    d_t1 (sigma u_z^2): the time derivative of sigma u^2 is taken as
    2 sigma u d_t1 u, with sigma d_t1 u = d_t1 (sigma u) - u d_t1 sigma; and
    d_t1 sigma = theta d_t1 (sigma - P) with P / sigma held fixed, so that
    theta = sigma / (sigma - P), which equals the printed
    1 + [(eps/P + 1) gamma^2 - 1]^-1. Returns (C, parts) with C = D_7 minus
    the target residual, and the symbolic pieces used by the checks."""
    sp = pytest.importorskip("sympy")
    y = sp.symbols("y")
    s = sp.Function("sigma")(y)
    u = sp.Function("u")(y)
    P = s * (1 - u ** 2) / 4  # P = eps/3 with sigma = (eps + P) gamma^2
    gam = 1 / sp.sqrt(1 - u ** 2)
    c2 = sp.Rational(1, 3)
    E = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
    W = [sp.Rational(4, 9)] + [sp.Rational(1, 9)] * 4 + [sp.Rational(1, 36)] * 4

    def geq(a):
        eu = E[a][1] * u
        if a == 0:
            return W[0] * s * (sp.Rational(9, 4) - P * (5 + 9 * c2) / (4 * s * c2)
                               - u ** 2 / (2 * c2))
        return W[a] * s * (P / (s * c2) + eu / c2 + eu ** 2 / (2 * c2 ** 2) - u ** 2 / (2 * c2))

    g = [geq(a) for a in range(9)]
    r7 = [ex * ex - ey * ey for ex, ey in E]
    m7 = sum(r * q for r, q in zip(r7, g))
    F7 = sum(r * E[a][1] * g[a] for a, r in enumerate(r7))
    En = sum(g)
    Mo = sum(E[a][1] * g[a] for a in range(9))
    Pyy = sum(E[a][1] ** 2 * g[a] for a in range(9))
    dt_E = -sp.diff(Mo, y)
    dt_M = -sp.diff(Pyy, y)
    theta = s / En
    dt_s = theta * dt_E
    s_dt_u = dt_M - u * dt_s
    dt_m7 = -2 * u * s_dt_u  # m7_eq = -sigma u^2 (checked by the next test)
    D7 = dt_m7 + sp.diff(F7, y)
    target = -2 * c2 * s / gam * sp.diff(gam * u, y)
    C = D7 - target
    S, U, dS, dU = sp.symbols("S U dS dU")
    flat = C.subs({sp.Derivative(s, y): dS, sp.Derivative(u, y): dU}).subs({s: S, u: U})
    parts = {"sp": sp, "y": y, "s": s, "u": u, "P": P, "gam": gam, "c2": c2, "m7": m7,
             "F7": F7, "E": En, "M": Mo, "Pyy": Pyy, "theta": theta, "C": C,
             "args": (S, U, dS, dU)}
    return sp.lambdify((S, U, dS, dU), sp.simplify(flat), "numpy"), parts


def test_expansion_route_reproduces_eq38():
    """The moments the derivation uses are those of Eqs. (32)-(33), theta is
    the printed one, and the route gives the printed C_7 to all orders in u
    (with the sign of this basis' row 7)."""
    _, d = _c7_from_the_expansion()
    sp, y, s, u, P, gam, c2 = (d[k] for k in ("sp", "y", "s", "u", "P", "gam", "c2"))
    assert sp.simplify(d["m7"] + s * u ** 2) == 0
    assert sp.simplify(d["F7"] + (1 - c2) * s * u) == 0
    assert sp.simplify(d["E"] - (s - P)) == 0
    assert sp.simplify(d["M"] - s * u) == 0
    assert sp.simplify(d["Pyy"] - (s * u ** 2 + P)) == 0
    eps = 3 * P
    theta_printed = 1 + 1 / ((eps / P + 1) * gam ** 2 - 1)
    assert sp.simplify(d["theta"] - theta_printed) == 0
    dd = lambda q: sp.diff(q, y)  # noqa: E731
    printed = 2 * (u * dd(c2 * s - P) - c2 * s / gam * u * dd(gam) - u * dd(s * u ** 2)
                   + u ** 2 * theta_printed * dd(s * u))
    assert sp.simplify(sp.expand(d["C"] + printed)) == 0


def _tube_fields(orc, L, umax, tau_v):
    """One-step runs of a smooth periodic 1 x L flow along y with and without
    the correction: the fields the corrected step differentiates, and the
    change of m_7 the correction made, divided by (1 - s_v / 2)."""
    k = 2 * np.pi / L
    y = np.arange(L)
    runs = {}
    for corr in (0, 1):
        prob = _tube(L, correction=corr, tau_v=tau_v)
        prob.eps[0, :, 0] = 1.0 + 0.3 * np.cos(k * y + 0.3)
        prob.n[0, :, 0] = 1.0 + 0.2 * np.sin(k * y)
        prob.u[1, 0, :, 0] = umax * (0.8 * np.sin(k * y) + 0.2 * np.sin(2 * k * y + 1.0))
        runs[corr] = orc.run(prob, 1)
    # collision conserves N, E, M: the fields of the uncorrected state after
    # one step are those of the pulled populations both runs collided
    F = runs[0].fields()
    M = orc.d2q9_tables()["M"]
    dm7 = (M @ (runs[1].g - runs[0].g).reshape(9, L))[7] / (1.0 - 0.5 / tau_v)
    eps, P, gam = F["eps"][0, :, 0], F["P"][0, :, 0], F["gamma"][0, :, 0]
    uy = F["u"][1, 0, :, 0]
    sig = (eps + P) * gam * gam
    cd = lambda a: 0.5 * (np.roll(a, -1) - np.roll(a, 1))  # noqa: E731
    return dm7, sig, uy, cd(sig), cd(uy)


@pytest.mark.parametrize("umax", [0.3, 0.55])
def test_correction_equals_the_expansion_at_every_order(orc, umax):
    """Pins every term of Eq. (38), the gamma term and theta included: the
    correction the oracle applies at each cell of a smooth tube equals the
    expansion of _c7_from_the_expansion, evaluated with central differences
    of sigma and u. What remains is the gap between a central difference of
    a product and the product rule, O(k^2): it falls fourfold from
    k = 2 pi / 1024 to 2 pi / 2048, and is below 1e-4 of the term there.
    Dropping the gamma term, or taking theta = 1 or its rest value 4/3,
    would move the result by more than 50 times that tolerance."""
    C, d = _c7_from_the_expansion()
    gaps = []
    for L in (1024, 2048):
        dm7, sig, uy, ds, du = _tube_fields(orc, L, umax, 1.7)
        want = C(sig, uy, ds, du)
        gaps.append(np.abs(dm7 - want).max() / np.abs(want).max())
    assert gaps[1] < 1e-4, gaps
    assert 3.5 < gaps[0] / gaps[1] < 4.5, gaps
    # each higher-order piece is far above the tolerance on this flow
    tol = 1e-4 * np.abs(want).max()
    gam2 = 1.0 / (1.0 - uy * uy)
    gamma_term = 2.0 / 3.0 * sig * gam2 * uy * uy * du  # 2 c_s^2 sigma gamma^-1 u dgamma
    theta = 4.0 * gam2 / (4.0 * gam2 - 1.0)
    theta_term = 2.0 * uy * uy * (uy * ds + sig * du)  # per unit of theta
    assert np.abs(gamma_term).max() > 50 * tol
    assert np.abs((theta - 1.0) * theta_term).max() > 50 * tol
    assert np.abs((theta - 4.0 / 3.0) * theta_term).max() > 50 * tol
