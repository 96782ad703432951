"""Seeded input generators: determinism, shapes and the stated ranges."""

import numpy as np

import workloads as wl


def test_random_modes_deterministic_and_scaled():
    a = wl.random_modes(16, 12, 10, seed=1211)
    b = wl.random_modes(16, 12, 10, seed=1211)
    c = wl.random_modes(16, 12, 10, seed=1212)
    assert np.array_equal(a.u, b.u) and np.array_equal(a.eps, b.eps)
    assert not np.array_equal(a.u, c.u)
    assert a.u.shape == (3, 10, 12, 16) and a.eps.shape == (10, 12, 16)
    assert abs(np.sqrt((a.u ** 2).sum(0)).max() - 0.1) < 1e-15
    assert abs(np.abs(a.eps - 1).max() - 0.05) < 1e-15
    assert abs(np.abs(a.n - 1).max() - 0.05) < 1e-15


def test_shock_tube_profile():
    p = wl.shock_tube(800)
    P = p.eps[:, 0, 0] / 3
    assert abs(P[0] - 1.0) < 1e-12 and abs(P[-1] - 0.41) < 1e-12
    assert abs(p.n[0, 0, 0] - 1.0) < 1e-12 and abs(p.n[-1, 0, 0] - 0.55) < 1e-12
    # the jump sits between cells 399 and 400
    assert P[399] > 0.5 * (1 + 0.41) > P[400]
    assert p.params.bc == (0, 0, 1) and (p.params.nx, p.params.ny, p.params.nz) == (1, 1, 800)


def test_tube_batch():
    tubes = wl.tube_batch()
    assert len(tubes) == 64
    L = [t.params.nz for t in tubes]
    assert min(L) >= 400 and max(L) <= 3200
    for t in tubes:
        p = t.params
        assert 0.6 <= p.tau_v <= 2.0 and 0.6 <= p.tau_eps <= 1.5
        assert 0.5 < p.tau_e <= p.tau_v
        assert abs(t.n - (t.eps / 3) ** 0.75).max() < 1e-15


def test_window_is_the_neighbourhood():
    prob = wl.random_modes(10, 9, 8, seed=3)
    sub, loc = wl.window(prob, (1, 4, 9), 2)
    assert sub.n.shape == (5, 5, 5)
    assert sub.n[loc] == prob.n[1, 4, 9]
    assert sub.n[0, 0, 0] == prob.n[(1 - 2) % 8, 2, (9 - 2) % 10]
