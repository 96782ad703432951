"""FP64 CPU oracle of the relativistic lattice Boltzmann step (ctypes binding).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``. The GPU package never imports
it, and it never imports the GPU package.

The arithmetic lives in ``rlb_oracle.cpp`` (built by ``oracle/build.py`` into
``oracle/liboracle.so``); this module only marshals numpy arrays.

Layout: populations are ``(Q, nz, ny, nx)`` float64 arrays (one for f, one
for g; Q = 19 for D3Q19, 9 for the D2Q9 model of Sec. V.A on nx x ny x 1
lattices); fields are ``(nz, ny, nx)`` and velocities ``(3, nz, ny, nx)``.
A problem selects its lattice with ``params.lattice`` ("d3q19" or "d2q9").
"""

from __future__ import annotations

import ctypes
import os
from typing import Dict, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")


class CParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("bc", ctypes.c_int32 * 3), ("tau_f", ctypes.c_double),
                ("tau_v", ctypes.c_double), ("tau_e", ctypes.c_double),
                ("tau_eps", ctypes.c_double), ("tau_q", ctypes.c_double),
                ("eta_s", ctypes.c_double), ("kappa", ctypes.c_double),
                ("dof", ctypes.c_double), ("a_f", ctypes.c_double), ("a_e", ctypes.c_double),
                ("a_eps", ctypes.c_double), ("a_q", ctypes.c_double),
                ("eos_gamma", ctypes.c_double), ("mass", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from oracle import build as _b
        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    D = ctypes.POINTER(ctypes.c_double)
    I = ctypes.POINTER(ctypes.c_int)
    P = ctypes.POINTER(CParams)
    lib.oracle_tables.argtypes = [I, D, D, D, D]
    lib.oracle_d2q9_tables.argtypes = [I, D, D]
    lib.oracle_d2q9_geq.argtypes = [ctypes.c_double, ctypes.c_double, D, D]
    lib.oracle_d2q9_feq.argtypes = [ctypes.c_double, ctypes.c_double, D, D]
    lib.oracle_d2q9_rates.argtypes = [P, D]
    lib.oracle_cell_taus.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, D]
    lib.oracle_d2q9_collide_cell.argtypes = [P, D, D, D, D]
    lib.oracle_d2q9_collide_cell.restype = ctypes.c_int
    lib.oracle_d2q9_init.argtypes = [P, D, D, D, D, D]
    lib.oracle_d2q9_step.argtypes = [P, ctypes.c_int32, D, D, ctypes.c_int32]
    lib.oracle_d2q9_step.restype = ctypes.c_int64
    lib.oracle_d2q9_fields.argtypes = [P, D, D, D, D, D, D, D, D]
    lib.oracle_d2q9_fields.restype = ctypes.c_int64
    lib.oracle_feq.argtypes = [ctypes.c_double, ctypes.c_double, D, D]
    lib.oracle_geq.argtypes = [ctypes.c_double, ctypes.c_double, D, D]
    lib.oracle_recover.argtypes = [ctypes.c_double, ctypes.c_double, D, D]
    lib.oracle_recover.restype = ctypes.c_int
    lib.oracle_recover_model.argtypes = [P, ctypes.c_double, ctypes.c_double, D, D]
    lib.oracle_recover_model.restype = ctypes.c_int
    lib.oracle_rates.argtypes = [P, D]
    lib.oracle_collide_cell.argtypes = [P, D, D, D, D]
    lib.oracle_collide_cell.restype = ctypes.c_int
    lib.oracle_init.argtypes = [P, D, D, D, D, D]
    lib.oracle_step.argtypes = [P, ctypes.c_int32, D, D]
    lib.oracle_step.restype = ctypes.c_int64
    lib.oracle_fields.argtypes = [P, D, D, D, D, D, D, D, D]
    lib.oracle_fields.restype = ctypes.c_int64
    lib.oracle_grad.argtypes = [P, ctypes.c_int32, D, D, D, D, D, D, D, D]
    lib.oracle_grad.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def is_d2q9(p) -> bool:
    return getattr(p, "lattice", "d3q19") == "d2q9"


def nvel(p) -> int:
    """Number of velocities of the lattice of ``p``."""
    return 9 if is_d2q9(p) else 19


def cparams(p) -> CParams:
    """Convert a ``workloads.Params`` (or any object with the same fields)."""
    c = CParams()
    c.nx, c.ny, c.nz = int(p.nx), int(p.ny), int(p.nz)
    for i in range(3):
        c.bc[i] = int(p.bc[i])
    c.tau_f, c.tau_v, c.tau_e = float(p.tau_f), float(p.tau_v), float(p.tau_e)
    c.tau_eps, c.tau_q = float(p.tau_eps), float(p.tau_q)
    c.eta_s = float(getattr(p, "eta_s", 0.0))
    c.kappa = float(getattr(p, "kappa", 1.0))
    c.dof = float(getattr(p, "dof", 16.0))
    for k in ("a_f", "a_e", "a_eps", "a_q", "eos_gamma", "mass"):
        setattr(c, k, float(getattr(p, k, 0.0)))
    return c


def general_eos(p) -> bool:
    g = float(getattr(p, "eos_gamma", 0.0))
    return (g != 0.0 and g != 4.0 / 3.0) or float(getattr(p, "mass", 0.0)) != 0.0


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def tables() -> Dict[str, np.ndarray]:
    """D3Q19 velocities, weights, moment basis M, M^-1 and squared row norms."""
    lib = _load()
    e = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    M = np.zeros((19, 19))
    Minv = np.zeros((19, 19))
    norms = np.zeros(19)
    lib.oracle_tables(e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _ptr(w), _ptr(M),
                      _ptr(Minv), _ptr(norms))
    return {"e": e.astype(np.int64), "w": w, "M": M, "Minv": Minv, "norms": norms}


def d2q9_tables() -> Dict[str, np.ndarray]:
    lib = _load()
    e = np.zeros((9, 2), dtype=np.int32)
    w = np.zeros(9)
    M = np.zeros((9, 9))
    lib.oracle_d2q9_tables(e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _ptr(w), _ptr(M))
    return {"e": e.astype(np.int64), "w": w, "M": M}


def d2q9_geq(sigma: float, P: float, u) -> np.ndarray:
    out = np.zeros(9)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    _load().oracle_d2q9_geq(float(sigma), float(P), _ptr(uu), _ptr(out))
    return out


def d2q9_feq(n: float, gamma: float, u) -> np.ndarray:
    out = np.zeros(9)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    _load().oracle_d2q9_feq(float(n), float(gamma), _ptr(uu), _ptr(out))
    return out


def feq(n: float, gamma: float, u) -> np.ndarray:
    out = np.zeros(19)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    _load().oracle_feq(float(n), float(gamma), _ptr(uu), _ptr(out))
    return out


def geq(eps: float, P: float, u) -> np.ndarray:
    out = np.zeros(19)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    _load().oracle_geq(float(eps), float(P), _ptr(uu), _ptr(out))
    return out


def recover(N: float, E: float, M) -> Tuple[bool, Dict[str, float]]:
    out = np.zeros(8)
    mm = np.ascontiguousarray(M, dtype=np.float64)
    ok = _load().oracle_recover(float(N), float(E), _ptr(mm), _ptr(out))
    keys = ["n", "eps", "P", "gamma", "ux", "uy", "uz", "sigma"]
    return bool(ok), dict(zip(keys, out.tolist()))


def recover_model(p, N: float, E: float, M) -> Tuple[bool, Dict[str, float]]:
    """Recovery under the equation of state of ``p`` (P = eps/3 or the
    general P = (Gamma - 1)(eps - m n))."""
    out = np.zeros(8)
    mm = np.ascontiguousarray(M, dtype=np.float64)
    cp = cparams(p)
    ok = _load().oracle_recover_model(ctypes.byref(cp), float(N), float(E), _ptr(mm), _ptr(out))
    keys = ["n", "eps", "P", "gamma", "ux", "uy", "uz", "sigma"]
    return bool(ok), dict(zip(keys, out.tolist()))


def rates(p) -> np.ndarray:
    """Diagonal of S (0 on the conserved rows)."""
    q = nvel(p)
    out = np.zeros(q)
    cp = cparams(p)
    fn = _load().oracle_d2q9_rates if q == 9 else _load().oracle_rates
    fn(ctypes.byref(cp), _ptr(out))
    return out


def cell_taus(p, n: float, P: float, gamma: float = 1.0, sigma=None) -> Dict[str, float]:
    """Relaxation times of a cell with fields (n, P, gamma, sigma); sigma
    defaults to the P = eps/3 value 4 P gamma^2."""
    out = np.zeros(5)
    if sigma is None:
        sigma = 4.0 * P * gamma * gamma
    cp = cparams(p)
    _load().oracle_cell_taus(ctypes.byref(cp), float(n), float(P), float(gamma), float(sigma),
                             _ptr(out))
    return dict(zip(["tau_f", "tau_v", "tau_e", "tau_eps", "tau_q"], out.tolist()))


def collide_cell(p, f, g):
    q = nvel(p)
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    assert f.shape == (q,) and g.shape == (q,)
    fo = np.zeros(q)
    go = np.zeros(q)
    cp = cparams(p)
    fn = _load().oracle_d2q9_collide_cell if q == 9 else _load().oracle_collide_cell
    ok = fn(ctypes.byref(cp), _ptr(f), _ptr(g), _ptr(fo), _ptr(go))
    return bool(ok), fo, go


class State:
    """Populations (f, g) of one lattice plus its parameters."""

    def __init__(self, params, f, g):
        self.params = params
        self.f = f
        self.g = g
        self.t = 0
        self.bad = 0

    @classmethod
    def init(cls, problem) -> "State":
        p = problem.params
        shape = (nvel(p), p.nz, p.ny, p.nx)
        f = np.zeros(shape)
        g = np.zeros(shape)
        cp = cparams(p)
        n0 = np.ascontiguousarray(problem.n, dtype=np.float64)
        e0 = np.ascontiguousarray(problem.eps, dtype=np.float64)
        u0 = np.ascontiguousarray(problem.u, dtype=np.float64)
        if is_d2q9(p):
            if p.nz != 1 or np.any(u0[2] != 0.0):
                raise ValueError("a D2Q9 lattice is nx x ny x 1 with u_z = 0")
            fn = _load().oracle_d2q9_init
        else:
            fn = _load().oracle_init
        fn(ctypes.byref(cp), _ptr(n0), _ptr(e0), _ptr(u0), _ptr(f), _ptr(g))
        return cls(p, f, g)

    def step(self, nsteps: int = 1) -> int:
        cp = cparams(self.params)
        if is_d2q9(self.params):
            corr = int(bool(getattr(self.params, "correction", 0)))
            if corr and general_eos(self.params):
                raise ValueError("the correction term is defined for P = eps/3")
            bad = _load().oracle_d2q9_step(ctypes.byref(cp), int(nsteps), _ptr(self.f),
                                           _ptr(self.g), corr)
        else:
            if getattr(self.params, "correction", 0):
                raise ValueError("the correction term of Eqs. (37)-(38) is a D2Q9 option")
            bad = _load().oracle_step(ctypes.byref(cp), int(nsteps), _ptr(self.f), _ptr(self.g))
        self.t += nsteps
        self.bad += int(bad)
        return int(bad)

    def fields(self):
        """n, eps, P, gamma, u (3 planes), sums[5], number of inadmissible cells."""
        p = self.params
        shape = (p.nz, p.ny, p.nx)
        n = np.zeros(shape)
        eps = np.zeros(shape)
        P = np.zeros(shape)
        gam = np.zeros(shape)
        u = np.zeros((3,) + shape)
        sums = np.zeros(5)
        cp = cparams(p)
        fn = _load().oracle_d2q9_fields if is_d2q9(p) else _load().oracle_fields
        bad = fn(ctypes.byref(cp), _ptr(self.f), _ptr(self.g), _ptr(n), _ptr(eps), _ptr(P),
                 _ptr(gam), _ptr(u), _ptr(sums))
        return {"n": n, "eps": eps, "P": P, "gamma": gam, "u": u, "sums": sums,
                "bad": int(bad)}


def run(problem, nsteps: int) -> State:
    st = State.init(problem)
    if nsteps:
        st.step(nsteps)
    return st


def grad(problem, nsteps: int, dL_du: np.ndarray, dL_deps: np.ndarray):
    """FP64 adjoint: (dL/d(tau_v, tau_e, tau_eps), dL/deps0, dL/du0). D3Q19 only."""
    p = problem.params
    if is_d2q9(p):
        raise ValueError("the adjoint oracle covers the D3Q19 model only")
    shape = (p.nz, p.ny, p.nx)
    dtau = np.zeros(3)
    de0 = np.zeros(shape)
    du0 = np.zeros((3,) + shape)
    cp = cparams(p)
    args = [np.ascontiguousarray(a, dtype=np.float64)
            for a in (problem.n, problem.eps, problem.u, dL_du, dL_deps)]
    code = _load().oracle_grad(ctypes.byref(cp), int(nsteps), *[_ptr(a) for a in args],
                               _ptr(dtau), _ptr(de0), _ptr(du0))
    if code != 0:
        raise ValueError("the adjoint oracle covers fixed relaxation times only")
    return dtau, de0, du0
