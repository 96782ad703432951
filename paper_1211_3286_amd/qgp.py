"""Quark-gluon-plasma units and relaxation times from eta/s (host side).

The paper runs its shock tubes (Sec. III.B, V.B) in lattice units fixed by
two statements: t = 400 dt is 3.2 fm/c, so dt = dx = 0.008 fm (c = 1); and a
temperature of 350 MeV is 0.0314, which fixes the energy unit (about
11.15 GeV). Pressures convert with dx^3 / energy unit (5.43 GeV/fm^3 is then
2.494e-7, the printed 2.495e-7), particle densities with dx^3, and
n = P / T for the ideal gas of the initial states.

Relaxation times follow from the ratio eta/s (Sec. III.B): the entropy
density is s = 4n - n ln(lambda), lambda = n / n_eq, n_eq = d_G T^3 / pi^2
(d_G = 16 for gluons), and the viscosity relation after Eq. (10),
eta = (tau - 1/2) c_s^2 (eps + P) gamma, gives
tau = 1/2 + kappa (eta/s) s / (c_s^2 (eps + P) gamma), which the kernels
evaluate per cell (rlb_params.eta_over_s). kappa is the transformation of the
shear viscosity the model needs for (1+1)-dimensional flows: 1 for the plain
relation of Sec. III, 2/3 for the BGK model in 3D (Sec. IV: 2 eta in place of
4 eta / 3) and 4/3 for the D2Q9 MRT model with a small bulk viscosity
(Sec. V.A, Eq. 36 with D = 2); this module holds those constants and the unit
conversions only.
"""

from __future__ import annotations

DX_FM = 3.2 / 400.0  # lattice spacing and time step, fm (and fm/c)
E_UNIT_GEV = 0.350 / 0.0314  # energy unit: 350 MeV is 0.0314
DOF_GLUONS = 16.0
CS2 = 1.0 / 3.0

KAPPA_PLAIN = 1.0
KAPPA_D3Q19_BGK_1D = 2.0 / 3.0
KAPPA_D2Q9_MRT = 4.0 / 3.0


def lattice_temperature(T_MeV: float) -> float:
    return T_MeV * 1e-3 / E_UNIT_GEV


def lattice_pressure(P_GeV_per_fm3: float) -> float:
    return P_GeV_per_fm3 * DX_FM ** 3 / E_UNIT_GEV


def lattice_density(n_per_fm3: float) -> float:
    return n_per_fm3 * DX_FM ** 3


def time_fm(steps: float) -> float:
    return steps * DX_FM
