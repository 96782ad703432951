"""Seeded synthetic inputs shaped like the paper's relativistic flow problems.

This module is shared by the GPU path and the FP64 oracle: it only draws and
lays out initial fields and relaxation times. It holds none of the lattice
Boltzmann arithmetic (no equilibria, moments, recovery or collision).

Conventions
-----------
* A lattice of ``nx * ny * nz`` cells is stored C-ordered as ``(nz, ny, nx)``
  (x fastest). Vector fields are ``(3, nz, ny, nx)``.
* Every field is float64. The pressure values the problems are stated in are
  turned into energy density with the ideal ultra-relativistic equation of
  state the method runs with, P = eps / 3, so ``eps = 3 * P``.
* Boundary kinds: 0 = periodic, 1 = zero-gradient ("open").

Problems (the paper publishes no data set; these stand in for its
quark-gluon-plasma shock tubes of Sec. III.B and Sec. V.B and for the blast
problem class the model was built for):

``shock_tube``     quasi-1D Riemann problem on 1 x 1 x L cells (Sec. III.B).
``random_modes``   3D periodic smooth random flow (16 Fourier modes).
``tube_batch``     64 ragged shock tubes with per-tube relaxation times.
``shear_vortex``   2D periodic shear wave + Taylor-Green vortex (adjoint).
``blast``          3D spherical blast with an outward velocity shell.
``blast_disk``     its 2D analogue for the D2Q9 model.
``qgp_tube_2d``    the 4 x 800 D2Q9 shock tube of Sec. V.B, Cases A-D.
``qgp_tube_3d``    the 1 x 1 x 800 D3Q19 shock tube of Sec. III.B at given eta/s.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Tuple

import numpy as np

PERIODIC = 0
ZERO_GRADIENT = 1


@dataclasses.dataclass
class Params:
    """Lattice size, boundary kinds and relaxation times of one lattice."""

    nx: int
    ny: int
    nz: int
    bc: Tuple[int, int, int] = (PERIODIC, PERIODIC, PERIODIC)
    tau_f: float = 0.9
    tau_v: float = 0.9
    tau_e: float = 0.9
    tau_eps: float = 0.9
    tau_q: float = 0.0  # <= 0: ghost moments relax with tau_v
    lattice: str = "d3q19"  # or "d2q9" (nx x ny x 1, velocities in the x-y plane)
    correction: int = 0  # D2Q9: 1 adds the C_7 term of Eqs. (37)-(38) (flow along y)
    # Relaxation times from eta/s per cell (Sec. III.B) when eta_s > 0: tau_v from
    # the local state, scaled by kappa; tau_x - 1/2 = a_x (tau_v - 1/2) where a_x > 0.
    eta_s: float = 0.0
    kappa: float = 1.0
    dof: float = 16.0  # degeneracy d_G of n_eq = d_G T^3 / pi^2 (gluons)
    a_f: float = 0.0
    a_e: float = 0.0
    a_eps: float = 0.0
    a_q: float = 0.0
    # Equation of state P = (Gamma - 1)(eps - m n); eos_gamma = 0 (or 4/3) with
    # mass = 0 is the paper's P = eps/3.
    eos_gamma: float = 0.0
    mass: float = 0.0

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz


@dataclasses.dataclass
class Problem:
    """Initial fields (float64) plus the lattice parameters."""

    params: Params
    n: np.ndarray
    eps: np.ndarray
    u: np.ndarray
    name: str = ""
    meta: Dict = dataclasses.field(default_factory=dict)


def _tanh_step(i: np.ndarray, center: float, width: float, left: float, right: float) -> np.ndarray:
    """left for i << center, right for i >> center, smoothed over ~2 cells."""
    s = 0.5 * (1.0 - np.tanh((i + 0.5 - center) / width))
    return right + (left - right) * s


def shock_tube(length: int = 800, P_L: float = 1.0, n_L: float = 1.0, P_R: float = 0.41,
               n_R: float = 0.55, width: float = 1.0, tau: float = 0.9,
               tau_f: float | None = None) -> Problem:
    """Quasi-1D Riemann problem at rest on a 1 x 1 x ``length`` lattice.

    The long axis is z with zero-gradient ends; the two transverse axes have
    one cell and are periodic. The jump sits between cells length/2 - 1 and
    length/2 and is smoothed with a tanh of width ``width`` cells.
    """
    z = np.arange(length, dtype=np.float64)
    P = _tanh_step(z, length / 2.0, width, P_L, P_R)
    n = _tanh_step(z, length / 2.0, width, n_L, n_R)
    shape = (length, 1, 1)
    prm = Params(1, 1, length, (PERIODIC, PERIODIC, ZERO_GRADIENT), tau_f if tau_f else tau,
                 tau, tau, tau)
    return Problem(prm, n.reshape(shape).copy(), (3.0 * P).reshape(shape).copy(),
                   np.zeros((3,) + shape), name=f"shock_tube_1x1x{length}")


def _mode_set(rng: np.random.Generator, n_modes: int, kmax: float, ndim: int):
    """Draw ``n_modes`` integer wave vectors with 1 <= |k| <= kmax."""
    ks = []
    r = int(math.floor(kmax))
    while len(ks) < n_modes:
        k = rng.integers(-r, r + 1, size=3)
        if ndim == 2:
            k[2] = 0
        kk = float(np.sqrt((k * k).sum()))
        if 1.0 <= kk <= kmax:
            ks.append(k)
    return np.array(ks, dtype=np.int64)


def _mode_sum(shape, ks, amps, phases):
    """sum_m amps[m] * cos(2 pi k_m . x / L + phase_m) on the (nz, ny, nx) grid.

    ``amps`` is (n_modes, ncomp). Returns (ncomp, nz, ny, nx). Evaluated as a
    product of 1D complex exponentials per axis.
    """
    nz, ny, nx = shape
    ncomp = amps.shape[1]
    out = np.zeros((ncomp,) + shape)
    x = np.arange(nx)
    y = np.arange(ny)
    z = np.arange(nz)
    for m in range(ks.shape[0]):
        kx, ky, kz = ks[m]
        ax = np.exp(2j * np.pi * ((kx * x) % nx) / nx)
        ay = np.exp(2j * np.pi * ((ky * y) % ny) / ny)
        az = np.exp(1j * (2 * np.pi * ((kz * z) % nz) / nz + phases[m]))
        plane = ay[:, None] * ax[None, :]
        wave = (az[:, None, None] * plane[None, :, :]).real
        for c in range(ncomp):
            out[c] += amps[m, c] * wave
    return out


def _noise(rng, shape, n_modes=16, kmax=4.0, ndim=3):
    ks = _mode_set(rng, n_modes, kmax, ndim)
    amps = rng.standard_normal((n_modes, 1))
    ph = rng.uniform(0.0, 2.0 * np.pi, n_modes)
    f = _mode_sum(shape, ks, amps, ph)[0]
    return f / np.abs(f).max()


def random_modes(nx: int = 256, ny: int | None = None, nz: int | None = None, seed: int = 1211,
                 umax: float = 0.1, amp: float = 0.05, n_modes: int = 16, kmax: float = 4.0,
                 tau_v: float = 0.8, tau_e: float = 0.55, tau_eps: float = 0.7,
                 tau_f: float = 0.8, bc=(PERIODIC, PERIODIC, PERIODIC)) -> Problem:
    """Smooth periodic random flow: 16 modes with integer |k| <= 4.

    u = sum of vector-amplitude cosine modes scaled to max|u| = umax;
    eps = 1 + amp * noise, n = 1 + amp * noise' with noise fields built the
    same way and normalised to max|noise| = 1.
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    shape = (nz, ny, nx)
    ndim = 2 if nz == 1 else 3
    rng = np.random.Generator(np.random.PCG64(seed))
    ks = _mode_set(rng, n_modes, kmax, ndim)
    amps = rng.standard_normal((n_modes, 3))
    if ndim == 2:
        amps[:, 2] = 0.0
    ph = rng.uniform(0.0, 2.0 * np.pi, n_modes)
    u = _mode_sum(shape, ks, amps, ph)
    speed = np.sqrt((u * u).sum(axis=0)).max()
    u *= umax / speed
    eps = 1.0 + amp * _noise(rng, shape, n_modes, kmax, ndim)
    n = 1.0 + amp * _noise(rng, shape, n_modes, kmax, ndim)
    prm = Params(nx, ny, nz, tuple(bc), tau_f, tau_v, tau_e, tau_eps)
    return Problem(prm, n, eps, u, name=f"random_modes_{nx}x{ny}x{nz}_seed{seed}")


def tube_batch(n_tubes: int = 64, seed: int = 3286, lmin: int = 400, lmax: int = 3200,
               ratio: Tuple[float, float] = (1.5, 5.0), tau_v: Tuple[float, float] = (0.6, 2.0),
               a: Tuple[float, float] = (0.05, 1.0), tau_eps: Tuple[float, float] = (0.6, 1.5),
               width: float = 1.0) -> List[Problem]:
    """Ragged batch of quasi-1D shock tubes (high-viscosity regime).

    Per tube: L ~ U{lmin..lmax}; P_L = 1, P_R = 1/r with r ~ U(ratio);
    n = P^(3/4); u = 0; tau_v ~ U(tau_v); tau_e = 1/2 + a (tau_v - 1/2) with
    a ~ U(a) (the paper's bulk/shear relaxation parameterisation of Cases C/D);
    tau_eps ~ U(tau_eps); tau_f = tau_v.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in range(n_tubes):
        L = int(rng.integers(lmin, lmax + 1))
        r = float(rng.uniform(*ratio))
        tv = float(rng.uniform(*tau_v))
        aa = float(rng.uniform(*a))
        te = 0.5 + aa * (tv - 0.5)
        tpe = float(rng.uniform(*tau_eps))
        z = np.arange(L, dtype=np.float64)
        P = _tanh_step(z, L / 2.0, width, 1.0, 1.0 / r)
        n = P ** 0.75
        shape = (L, 1, 1)
        prm = Params(1, 1, L, (PERIODIC, PERIODIC, ZERO_GRADIENT), tv, tv, te, tpe)
        out.append(Problem(prm, n.reshape(shape).copy(), (3.0 * P).reshape(shape).copy(),
                           np.zeros((3,) + shape), name=f"tube{b}_L{L}",
                           meta={"ratio": r, "a": aa}))
    return out


def shear_vortex(L: int = 512, seed: int = 1212, umax: float = 0.1, amp: float = 0.05,
                 tau_v: float = 0.8, tau_e: float = 0.55, tau_eps: float = 0.7,
                 tau_f: float = 0.8) -> Problem:
    """2D periodic L x L x 1 field: shear wave plus a Taylor-Green vortex.

    u_x = U0 sin(2 pi y / L) + sin(kx) cos(ky), u_y = -cos(kx) sin(ky) with
    k = 2 pi / L, scaled to max|u| = umax; eps = 1 + amp * noise; n = 1.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (1, L, L)
    k = 2.0 * np.pi / L
    x = np.arange(L)[None, None, :]
    y = np.arange(L)[None, :, None]
    u = np.zeros((3,) + shape)
    u[0] = 1.0 * np.sin(k * y) + np.sin(k * x) * np.cos(k * y)
    u[1] = -np.cos(k * x) * np.sin(k * y) + 0.0 * x
    u *= umax / np.sqrt((u * u).sum(axis=0)).max()
    eps = 1.0 + amp * _noise(rng, shape, ndim=2)
    n = np.ones(shape)
    prm = Params(L, L, 1, (PERIODIC, PERIODIC, PERIODIC), tau_f, tau_v, tau_e, tau_eps)
    return Problem(prm, n, eps, u, name=f"shear_vortex_{L}x{L}")


def perturbed_taus(base: Tuple[float, float, float], seed: int = 1212, rel: float = 0.05):
    """Target relaxation times tau'_k = tau_k + rel (tau_k - 1/2) z_k, z ~ N(0, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    z = rng.standard_normal(3)
    return tuple(float(t + rel * (t - 0.5) * zz) for t, zz in zip(base, z))


def target_noise(shape, seed: int = 1212, rel: float = 0.01):
    """Per-cell standard normal draws for the 1 % target noise: (4, *shape)."""
    rng = np.random.Generator(np.random.PCG64(seed + 11))
    return rng.standard_normal((4,) + tuple(shape))


def blast(L: int = 512, radius: float | None = None, shell: float | None = None,
          seed: int = 1213, P_in: float = 10.0, P_out: float = 0.1, umax: float = 0.6,
          tau_v: float = 0.9, tau_e: float = 0.62, tau_eps: float = 0.8,
          tau_f: float | None = None, width: float = 1.0) -> Problem:
    """Moderately relativistic 3D blast on an L^3 lattice with zero-gradient faces.

    P = P_in inside a sphere of radius L/8 (64 at L = 512), P_out outside
    (tanh width 1); n = P^(3/4); outward velocity shell
    u = umax exp(-((r - R)/w)^2)(1 + 0.1 noise) r_hat, w = R/8, rescaled to
    max|u| = umax.
    """
    R = L / 8.0 if radius is None else radius
    w = R / 8.0 if shell is None else shell
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (L, L, L)
    c = (L - 1) / 2.0
    ax = np.arange(L, dtype=np.float64) - c
    r = np.sqrt(ax[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2)
    P = P_out + (P_in - P_out) * 0.5 * (1.0 - np.tanh((r - R) / width))
    n = P ** 0.75
    mag = np.exp(-((r - R) / w) ** 2) * (1.0 + 0.1 * _noise(rng, shape))
    rs = np.where(r > 0, r, 1.0)
    del r
    u = np.empty((3,) + shape)
    u[0] = mag * ax[None, None, :] / rs
    u[1] = mag * ax[None, :, None] / rs
    u[2] = mag * ax[:, None, None] / rs
    del mag, rs
    u *= umax / np.sqrt((u * u).sum(axis=0)).max()
    tf = tau_v if tau_f is None else tau_f
    prm = Params(L, L, L, (ZERO_GRADIENT,) * 3, tf, tau_v, tau_e, tau_eps)
    return Problem(prm, n, 3.0 * P, u, name=f"blast_{L}x{L}x{L}")


def blast_disk(L: int = 136, radius: float | None = None, seed: int = 1214, P_in: float = 10.0,
               P_out: float = 0.1, umax: float = 0.6, tau_v: float = 0.9, tau_e: float = 0.62,
               tau_eps: float = 0.8, tau_f: float | None = None, correction: int = 0) -> Problem:
    """The 2D analogue of ``blast`` for the D2Q9 model on an L x L lattice
    with zero-gradient faces: P = P_in inside a disk of radius L/8, P_out
    outside (tanh width 1), n = P^(3/4), an outward velocity ring of width R/8
    rescaled to max|u| = umax. At umax = 0.6 the ring's leading edge turns
    cells inadmissible within a few steps."""
    R = L / 8.0 if radius is None else radius
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (1, L, L)
    c = (L - 1) / 2.0
    ax = np.arange(L, dtype=np.float64) - c
    r = np.sqrt(ax[:, None] ** 2 + ax[None, :] ** 2)[None]
    P = P_out + (P_in - P_out) * 0.5 * (1.0 - np.tanh(r - R))
    n = P ** 0.75
    mag = np.exp(-((r - R) / (R / 8.0)) ** 2) * (1.0 + 0.1 * _noise(rng, shape, ndim=2))
    rs = np.where(r > 0, r, 1.0)
    u = np.zeros((3,) + shape)
    u[0] = mag * ax[None, None, :] / rs
    u[1] = mag * ax[None, :, None] / rs
    u *= umax / np.sqrt((u * u).sum(axis=0)).max()
    tf = tau_v if tau_f is None else tau_f
    prm = Params(L, L, 1, (ZERO_GRADIENT, ZERO_GRADIENT, PERIODIC), tf, tau_v, tau_e, tau_eps)
    prm.lattice = "d2q9"
    prm.correction = correction
    return Problem(prm, n, 3.0 * P, u, name=f"blast_disk_{L}x{L}")


# Initial states of the quark-gluon-plasma shock tubes in lattice units
# (Sec. III.B and the moderately relativistic case of Sec. V.B): pressure
# left / right of the membrane and temperature left / right; n = P / T.
QGP_WEAK = {"P_L": 2.495e-7, "P_R": 1.023e-7, "T_L": 0.0314, "T_R": 0.0314}
QGP_MODERATE = {"P_L": 2.495e-7, "P_R": 1.557e-8, "T_L": 0.0359, "T_R": 0.018}


def case_taus(case: str, tau_v: float, a: float) -> Dict[str, float]:
    """Relaxation times of the four MRT cases of Sec. V.B, with
    tau_x - 1/2 = a (tau_v - 1/2) for the reduced ones:
    A: tau_e = tau_eps = tau_q = tau_v;  B: tau_q reduced;
    C: tau_e reduced;                    D: tau_e and tau_eps reduced."""
    red = 0.5 + a * (tau_v - 0.5)
    t = {"tau_v": tau_v, "tau_e": tau_v, "tau_eps": tau_v, "tau_q": tau_v}
    if case == "B":
        t["tau_q"] = red
    elif case == "C":
        t["tau_e"] = red
    elif case == "D":
        t["tau_e"] = red
        t["tau_eps"] = red
    elif case != "A":
        raise ValueError(f"unknown case {case!r}")
    return t


def case_ratios(case: str, a: float) -> Dict[str, float]:
    """The Cases of Sec. V.B for relaxation times set per cell from eta/s:
    tau_x - 1/2 = a_x (tau_v - 1/2) with a_x = a for the reduced ones, 1 else."""
    r = {"a_e": 1.0, "a_eps": 1.0, "a_q": 1.0}
    reduced = {"A": (), "B": ("a_q",), "C": ("a_e",), "D": ("a_e", "a_eps")}
    if case not in reduced:
        raise ValueError(f"unknown case {case!r}")
    for k in reduced[case]:
        r[k] = a
    return r


def qgp_tube_2d(case: str = "D", a: float = 1.0 / 20.0, tau_v: float = 100.0,
                tau_f: float = 0.6, nx: int = 4, length: int = 800, moderate: bool = False,
                width: float = 1.0, correction: bool = False, eta_s: float = 0.0,
                kappa: float = 4.0 / 3.0) -> Problem:
    """D2Q9 shock tube of Sec. V.B on nx x length x 1 cells.

    x is periodic (nx = 4 cells), the long axis y stands for the paper's z
    and has zero-gradient ends; the membrane sits between cells length/2 - 1
    and length/2 (tanh of width ``width``). Weak case: P_L, P_R of Sec. III.B
    at T = 0.0314; ``moderate``: the moderately relativistic case (P_R =
    1.557e-8, T_L / T_R = 0.0359 / 0.018). n = P / T, u = 0. Relaxation times
    from ``case_taus``; tau_v = 100 stands for the paper's value of roughly 100.
    ``correction`` adds the C_7 term of Eqs. (37)-(38) (the corrected runs).
    ``eta_s`` > 0: relaxation times per cell from eta/s (scaled by ``kappa``,
    4/3 for this D2Q9 model), with the case's ratios; tau_v then only serves
    as the fallback for cells without a temperature.
    """
    st = QGP_MODERATE if moderate else QGP_WEAK
    y = np.arange(length, dtype=np.float64)
    P = _tanh_step(y, length / 2.0, width, st["P_L"], st["P_R"])
    T = _tanh_step(y, length / 2.0, width, st["T_L"], st["T_R"])
    n = P / T
    shape = (1, length, nx)
    t = case_taus(case, tau_v, a)
    prm = Params(nx, length, 1, (PERIODIC, ZERO_GRADIENT, PERIODIC), tau_f, t["tau_v"],
                 t["tau_e"], t["tau_eps"], t["tau_q"], "d2q9", int(bool(correction)))
    if eta_s > 0.0:
        prm.eta_s, prm.kappa = eta_s, kappa
        for k, v in case_ratios(case, a).items():
            setattr(prm, k, v)
    ones = np.ones((1, 1, nx))
    return Problem(prm, (n[None, :, None] * ones).copy(), (3.0 * P[None, :, None] * ones).copy(),
                   np.zeros((3,) + shape),
                   name=f"qgp_tube_2d_{nx}x{length}_case{case}" + ("_moderate" if moderate else "")
                   + ("_c7" if correction else "") + (f"_eta_s{eta_s}" if eta_s > 0 else ""),
                   meta={"case": case, "a": a})


def qgp_tube_3d(eta_s: float = 0.1, tau_f: float | str = "tau_g", length: int = 800,
                width: float = 1.0, kappa: float = 1.0) -> Problem:
    """D3Q19 shock tube of Sec. III.B on 1 x 1 x length cells, relaxation
    times per cell from eta/s (all g rates tied to tau_v, the BGK limit of the
    MRT). ``tau_f``: "tau_g" ties tau_f to the local tau_g, a number fixes it
    (the paper's three choices are tau_g, 1.0 and 0.6)."""
    st = QGP_WEAK
    z = np.arange(length, dtype=np.float64)
    P = _tanh_step(z, length / 2.0, width, st["P_L"], st["P_R"])
    T = _tanh_step(z, length / 2.0, width, st["T_L"], st["T_R"])
    n = P / T
    shape = (length, 1, 1)
    tg = 1.0  # fixed values: only a fallback for cells without a temperature
    tied = tau_f == "tau_g"
    prm = Params(1, 1, length, (PERIODIC, PERIODIC, ZERO_GRADIENT), tg if tied else float(tau_f),
                 tg, tg, tg, 0.0, eta_s=eta_s, kappa=kappa, a_f=1.0 if tied else 0.0,
                 a_e=1.0, a_eps=1.0)
    return Problem(prm, n.reshape(shape).copy(), (3.0 * P).reshape(shape).copy(),
                   np.zeros((3,) + shape),
                   name=f"qgp_tube_3d_1x1x{length}_eta_s{eta_s}_tau_f_{tau_f}")


def uniform(nx: int, ny: int, nz: int, n: float = 1.0, eps: float = 1.0,
            u=(0.0, 0.0, 0.0), **tau) -> Problem:
    """A uniform state (every cell identical)."""
    shape = (nz, ny, nx)
    uu = np.empty((3,) + shape)
    for c in range(3):
        uu[c] = u[c]
    prm = Params(nx, ny, nz, tau.pop("bc", (PERIODIC,) * 3), **tau)
    return Problem(prm, np.full(shape, n), np.full(shape, eps), uu, name="uniform")


def window(problem: Problem, center: Tuple[int, int, int], half: int):
    """Cut the neighbourhood of ``center`` (z, y, x) that decides it after ``half`` steps.

    Returns (sub_problem, local_center). Periodic axes wrap (an axis shorter
    than 2*half+1 is taken whole); zero-gradient axes are cut at the real
    boundary, where the sub-lattice keeps the zero-gradient rule.
    """
    prm = problem.params
    dims = (prm.nz, prm.ny, prm.nx)
    bcs = (prm.bc[2], prm.bc[1], prm.bc[0])
    idx = []
    loc = []
    sub_bc = []
    for a in range(3):
        N = dims[a]
        c = center[a]
        if 2 * half + 1 >= N:
            idx.append(np.arange(N))
            loc.append(c)
            sub_bc.append(bcs[a])
        elif bcs[a] == PERIODIC:
            idx.append((c + np.arange(-half, half + 1)) % N)
            loc.append(half)
            sub_bc.append(ZERO_GRADIENT)
        else:
            lo = max(0, c - half)
            hi = min(N - 1, c + half)
            idx.append(np.arange(lo, hi + 1))
            loc.append(c - lo)
            sub_bc.append(ZERO_GRADIENT)
    iz, iy, ix = np.ix_(*idx)
    sub = dataclasses.replace(prm, nx=len(idx[2]), ny=len(idx[1]), nz=len(idx[0]),
                              bc=(sub_bc[2], sub_bc[1], sub_bc[0]))
    u = np.stack([problem.u[c][iz, iy, ix] for c in range(3)])
    return (Problem(sub, problem.n[iz, iy, ix].copy(), problem.eps[iz, iy, ix].copy(), u,
                    name=problem.name + "_window"), tuple(loc))
