"""Oracle pins: recovery of (n, eps, P, gamma, u) from the sums of Eq. (10).

The pins build the sums straight from the definitions of Eq. (10),
n gamma, (eps + P) gamma^2 - P and (eps + P) gamma^2 u with P = eps/3,
and check that the oracle returns the fields they came from; an independent
bisection on the two defining equations covers states the round trip does not.
"""

import numpy as np
import pytest


def _sums(n, eps, u):
    P = eps / 3.0
    gam = 1.0 / np.sqrt(1.0 - u @ u)
    sigma = (eps + P) * gam * gam
    return n * gam, sigma - P, sigma * u


@pytest.mark.parametrize("umax", [1e-9, 0.1, 0.6, 0.95, 0.999])
def test_round_trip(orc, umax):
    rng = np.random.default_rng(10)
    for _ in range(40):
        u = rng.normal(size=3)
        u *= umax / np.linalg.norm(u) * rng.uniform(0.5, 1.0)
        n = rng.uniform(0.01, 5.0)
        eps = rng.uniform(1e-3, 20.0)
        N, E, M = _sums(n, eps, u)
        ok, F = orc.recover(N, E, M)
        assert ok
        gam = 1.0 / np.sqrt(1.0 - u @ u)
        # conditioning of gamma grows like gamma^2 near the light cone
        tol = 4e-15 * gam * gam
        assert abs(F["eps"] - eps) <= tol * eps
        assert abs(F["P"] - eps / 3) <= tol * eps
        assert abs(F["n"] - n) <= tol * n
        assert abs(F["gamma"] - gam) <= tol * gam
        got = np.array([F["ux"], F["uy"], F["uz"]])
        assert np.abs(got - u).max() <= tol * max(np.linalg.norm(u), 1e-300)


def test_bisection_agrees(orc):
    """Solve E = sigma - sigma(1 - v^2)/4, |M| = sigma v by bisection on v."""
    rng = np.random.default_rng(11)
    for _ in range(30):
        E = rng.uniform(0.1, 5.0)
        Mabs = rng.uniform(0.0, 0.999) * E
        dirn = rng.normal(size=3)
        dirn /= np.linalg.norm(dirn)

        def resid(v):  # |M|(v) - |M| along the E-constraint: sigma = E / (1 - (1 - v^2)/4)
            sigma = E / (1.0 - (1.0 - v * v) / 4.0)
            return sigma * v - Mabs

        lo, hi = 0.0, 1.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if resid(mid) > 0:
                hi = mid
            else:
                lo = mid
        v = 0.5 * (lo + hi)
        ok, F = orc.recover(1.0, E, Mabs * dirn)
        assert ok
        got = np.array([F["ux"], F["uy"], F["uz"]])
        assert abs(np.linalg.norm(got) - v) < 1e-13
        sigma = E / (1.0 - (1.0 - v * v) / 4.0)
        assert abs(F["sigma"] - sigma) < 1e-12 * sigma
        assert abs(F["eps"] - 0.75 * sigma * (1 - v * v)) < 1e-12 * sigma


@pytest.mark.parametrize("E,M", [(0.0, (0.0, 0.0, 0.0)), (-1.0, (0.0, 0.0, 0.0)),
                                 (1.0, (1.0, 0.0, 0.0)), (1.0, (0.6, 0.6, 0.6)),
                                 (float("nan"), (0.0, 0.0, 0.0)), (1.0, (float("nan"), 0, 0)),
                                 (float("inf"), (0.0, 0.0, 0.0))])
def test_inadmissible(orc, E, M):
    ok, _ = orc.recover(1.0, E, np.array(M, dtype=float))
    if np.isinf(E):
        return  # inf passes E > 0 and |M| < E; nothing finite to compare
    assert not ok


def test_rest_state(orc):
    ok, F = orc.recover(2.0, 3.0, np.zeros(3))
    assert ok
    assert F["ux"] == F["uy"] == F["uz"] == 0.0
    assert F["gamma"] == 1.0
    assert abs(F["eps"] - 3.0) < 1e-15 and abs(F["P"] - 1.0) < 1e-15
    assert F["n"] == 2.0
