"""GPU parity: the HIP step (both dispatch paths, both precisions) against the
FP64 oracle, element by element, on seeded inputs that span several tiles and
ragged tails; plus the properties that hold at any size.

Tolerances (max-norm relative, max|a - b| / max|b|):
  FP64 populations and fields: 1e-12 (rounding-order differences only).
  FP32 populations: 1e-5 (the accuracy bar for the FP32 form).
"""

import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_helpers import compare, gpu_run, gpu_state, relmax, say

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
TOL = {FP64: 1e-12, FP32: 1e-5}

SHAPES = [
    # (nx, ny, nz, bc): lattice path (>= 16384 cells) and persistent path
    (37, 29, 23, (0, 0, 0)),
    (70, 33, 9, (1, 0, 1)),
    (13, 11, 7, (0, 1, 0)),
    (40, 9, 18, (1, 1, 1)),
    (300, 1, 60, (0, 0, 1)),
]


# Conserved sums of FP32-stored populations against the oracle's FP64 ones.
# Storing a population in FP32 rounds it by at most 2^-24 (6.0e-8) of itself,
# and the populations here are positive, so each sum of the stored values
# differs from the FP64 sum by at most 2^-24 of the largest sum: the bound
# is that, with 1.7x for the FP64 summation orders. Conservation over time
# (the GPU's sums against its own initial sums) has its own 1e-10 bar.
FP32_SUMS = 1e-7


def _problem(nx, ny, nz, bc, seed=7):
    return wl.random_modes(nx, ny, nz, seed=seed, umax=0.2, amp=0.1, tau_v=0.8, tau_e=0.55,
                           tau_eps=0.7, tau_f=0.63, bc=bc)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_init_and_export_match_oracle(prec):
    prob = _problem(37, 29, 23, (0, 0, 0))
    say("init/export", prob.name, "prec", prec)
    sim = gpu_run(prob, 0, prec)
    (gs,), sums, bad = gpu_state(sim, prob)
    st = oracle.State.init(prob)
    F = st.fields()
    err = compare(gs, st, F)
    tol = 1e-14 if prec == FP64 else 1e-7
    assert err["f"] < tol and err["g"] < tol, err
    # fields round-trip to the inputs
    ftol = 1e-13 if prec == FP64 else 1e-6
    assert relmax(gs["eps"], prob.eps) < ftol
    assert relmax(gs["n"], prob.n) < ftol
    assert np.abs(gs["u"] - prob.u).max() < ftol
    assert relmax(sums, F["sums"]) < (1e-13 if prec == FP64 else FP32_SUMS)
    assert bad == 0


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s[:3])) + f"_bc{s[3]}")
def test_step_matches_oracle(prec, shape):
    nx, ny, nz, bc = shape
    prob = _problem(nx, ny, nz, bc)
    T = 25
    say("step", prob.name, "bc", bc, "prec", prec, "steps", T)
    sim = gpu_run(prob, T, prec)
    say("  kernel", sim.kernel_name)
    (gs,), sums, bad = gpu_state(sim, prob)
    st = oracle.run(prob, T)
    F = st.fields()
    err = compare(gs, st, F)
    say("  errors", err)
    assert bad == 0 and st.bad == 0
    assert err["f"] < TOL[prec] and err["g"] < TOL[prec], err
    assert err["eps"] < TOL[prec] and err["n"] < TOL[prec] and err["u"] < TOL[prec], err
    assert relmax(sums, F["sums"]) < (1e-13 if prec == FP64 else FP32_SUMS)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_every_lattice_variant_is_identical(prec):
    """Block shape and cells-per-thread change the schedule, never a cell's
    arithmetic: every variant gives bit-identical populations."""
    import paper_1211_3286_amd as rlb
    prob = _problem(70, 33, 9, (1, 0, 1))
    ref = None
    sim0 = rlb.from_problems(prob, precision=prec)
    names = sim0.variants()
    for v, name in enumerate(names):
        say("variant", v, name, "prec", prec)
        sim = rlb.from_problems(prob, precision=prec)
        sim.variant = v
        sim.step(6)
        f, g = sim.populations()
        cur = (f.cpu().numpy(), g.cpu().numpy())
        if ref is None:
            ref = cur
            st = oracle.run(prob, 6)
            assert relmax(cur[0].reshape(st.f.shape), st.f) < TOL[prec]
        else:
            assert np.array_equal(cur[0], ref[0]) and np.array_equal(cur[1], ref[1]), name
        sim.close()


def test_tune_keeps_state_and_picks_a_variant():
    import paper_1211_3286_amd as rlb
    prob = _problem(70, 33, 9, (0, 0, 0))
    a = rlb.from_problems(prob, precision=FP32)
    b = rlb.from_problems(prob, precision=FP32)
    res = a.tune(trial_steps=3)
    say("tune", res)
    assert res["name"] in a.variants()
    assert all(v > 0 for v in res["ms_per_step"].values())
    a.step(4)
    b.step(4)
    fa, ga = a.populations()
    fb, gb = b.populations()
    assert bool((fa == fb).all()) and bool((ga == gb).all())
    assert a.steps == 4


def test_shock_tube_fp64_dumps():
    """1 x 1 x 800 relativistic Riemann problem, FP64, 2000 steps, fields
    compared with the oracle every 200 steps."""
    import paper_1211_3286_amd as rlb
    prob = wl.shock_tube(800, tau=0.9)
    sim = rlb.from_problems(prob, precision=FP64)
    st = oracle.State.init(prob)
    worst = 0.0
    for k in range(10):
        sim.step(200)
        st.step(200)
        (gs,), sums, bad = gpu_state(sim, prob)
        F = st.fields()
        err = compare(gs, st, F)
        worst = max(worst, err["f"], err["g"], err["eps"], err["n"], err["u"])
        say("  t", st.t, err)
        assert bad == 0 and st.bad == 0
    assert worst < 1e-12


def test_shock_tube_fp32_error_is_stated():
    import paper_1211_3286_amd as rlb
    prob = wl.shock_tube(800, tau=0.9)
    sim = rlb.from_problems(prob, precision=FP32)
    sim.step(2000)
    (gs,), sums, bad = gpu_state(sim, prob)
    st = oracle.run(prob, 2000)
    err = compare(gs, st, st.fields())
    say("shock tube FP32 vs FP64 oracle after 2000 steps:", err)
    assert err["f"] < 1e-5 and err["g"] < 1e-5


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_periodic_conservation(prec):
    prob = _problem(48, 40, 36, (0, 0, 0))
    sim = gpu_run(prob, 0, prec)
    s0 = sim.sums()
    sim.step(100)
    s1 = sim.sums()
    drift = np.abs(s1 - s0).max() / np.abs(s0[:2]).max()
    say("conservation drift", prec, drift, s0, s1)
    assert drift < (1e-13 if prec == FP64 else 1e-10)


@pytest.mark.parametrize("shape", [(37, 29, 23), (13, 11, 7)])
def test_fused_diagnostics(shape):
    """diag_every = 1: the step kernel's FP64 partial sums equal the oracle's
    conserved sums (periodic lattice)."""
    import paper_1211_3286_amd as rlb
    prob = _problem(*shape, (0, 0, 0))
    sim = rlb.from_problems(prob, precision=FP64, diag_every=1)
    sim.step(7)
    sim.moments()  # a field export in between leaves the diagnostics intact
    sums, step, bad = sim.diagnostics()
    st = oracle.run(prob, 7)
    assert step == 7 and bad == 0
    assert relmax(sums, st.fields()["sums"]) < 1e-13


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1)])
def test_uniform_state_is_stationary(prec, bc):
    import paper_1211_3286_amd as rlb
    for dims in ((40, 30, 20), (9, 8, 7)):
        prob = wl.uniform(*dims, n=1.3, eps=2.1, u=(0.3, -0.2, 0.1), bc=bc, tau_f=0.7,
                          tau_v=0.9, tau_e=0.6, tau_eps=1.1)
        sim = rlb.from_problems(prob, precision=prec)
        f0, g0 = [t.cpu().numpy() for t in sim.populations()]
        sim.step(10)
        f1, g1 = [t.cpu().numpy() for t in sim.populations()]
        tol = 1e-14 if prec == FP64 else 1e-6
        assert relmax(f1, f0) < tol and relmax(g1, g0) < tol


def test_inadmissible_cells_counted_like_the_oracle():
    """A 1000:1 expansion on 64 cells produces cells with E <= 0 or |M| >= E;
    both sides leave them uncollided and count them (FP64 decisions with a
    margin far above rounding). Next to near-vacuum cells the two sides'
    rounding differences are amplified, hence the looser population bound."""
    import paper_1211_3286_amd as rlb
    prob = wl.shock_tube(64, P_L=1.0, n_L=1.0, P_R=1e-3, n_R=1e-3 ** 0.75, tau=0.51)
    sim = rlb.from_problems(prob, precision=FP64)
    sim.step(14)
    (gs,), sums, bad = gpu_state(sim, prob)
    st = oracle.run(prob, 14)
    say("inadmissible: gpu", bad, "oracle", st.bad)
    assert bad == st.bad == 4
    assert relmax(gs["g"], st.g) < 1e-10 and relmax(gs["f"], st.f) < 1e-10


@pytest.mark.gpu
def test_inadmissible_count_over_many_blocks():
    """The lattice kernels count inadmissible cells in 256 slots picked by the
    block (one 128-byte line each) and the host sums them: on a 48^3 blast,
    whose inadmissible cells fall in several hundred blocks, every block shape
    gives the oracle's count (FP64)."""
    import paper_1211_3286_amd as rlb
    prob = wl.blast(48)
    T = 3
    st = oracle.run(prob, T)
    assert st.bad > 50
    sim = rlb.from_problems(prob, precision=FP64)
    names = sim.variants()
    sim.close()
    for v, name in enumerate(names):
        sim = rlb.from_problems(prob, precision=FP64)
        sim.variant = v
        sim.step(T)
        _, _, bad = gpu_state(sim, prob)
        say("  ", name, "gpu", bad, "oracle", st.bad)
        assert bad == st.bad, name
        sim.close()
