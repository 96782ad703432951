"""GPU parity of the D2Q9 MRT model (Sec. V.A, Eqs. 30-35) against the FP64
oracle: both dispatch paths (fused per-step lattice kernel, persistent
per-member kernel), both precisions, ragged tails and mixed boundaries; the
4 x 800 shock tube of Sec. V.B as a batch of Cases A-D over 400 steps; the
4096^2 benchmark lattice on sampled cells; conservation and variant identity.

Tolerances (max-norm relative): FP64 1e-12, FP32 1e-5.
"""

import re

import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_helpers import compare, gpu_run, gpu_state, relmax, say

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
TOL = {FP64: 1e-12, FP32: 1e-5}

SHAPES = [
    # (nx, ny, bc): >= 16384 cells take the lattice path, smaller the persistent one
    (131, 129, (0, 0, 0)),
    (300, 61, (1, 0, 0)),
    (37, 29, (0, 1, 0)),
    (1, 300, (0, 1, 0)),
    (300, 1, (1, 0, 0)),
    (70, 259, (1, 1, 0)),
]


def _problem(nx, ny, bc, seed=7, **kw):
    p = wl.random_modes(nx, ny, 1, seed=seed, umax=0.2, amp=0.1, tau_v=0.8, tau_e=0.55,
                        tau_eps=0.7, tau_f=0.63, bc=bc)
    p.params.lattice = "d2q9"
    p.params.tau_q = kw.get("tau_q", 1.1)
    return p


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}_bc{s[2]}")
def test_step_matches_oracle(prec, shape):
    nx, ny, bc = shape
    prob = _problem(nx, ny, bc)
    T = 25
    say("d2q9 step", prob.name, "bc", bc, "prec", prec)
    sim = gpu_run(prob, T, prec)
    say("  kernel", sim.kernel_name)
    (gs,), sums, bad = gpu_state(sim, prob)
    st = oracle.run(prob, T)
    F = st.fields()
    err = compare(gs, st, F)
    say("  errors", err)
    assert gs["f"].shape[0] == 9
    assert bad == 0 and st.bad == 0
    assert err["f"] < TOL[prec] and err["g"] < TOL[prec], err
    assert err["eps"] < TOL[prec] and err["n"] < TOL[prec] and err["u"] < TOL[prec], err
    assert np.abs(gs["u"][2]).max() == 0.0
    assert relmax(sums, F["sums"]) < (1e-13 if prec == FP64 else 1e-7)


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("shape", [(160, 130, (0, 1, 0)), (45, 38, (1, 0, 0))],
                         ids=["lattice", "persistent"])
def test_every_variant_is_identical(prec, shape):
    import paper_1211_3286_amd as rlb
    prob = _problem(*shape)
    ref = None
    sim0 = rlb.from_problems(prob, precision=prec)
    names = sim0.variants()
    sim0.close()
    for v in range(len(names)):
        sim = rlb.from_problems(prob, precision=prec)
        sim.variant = v
        try:
            sim.step(7)
        except rlb.RLBError as e:  # rounds whose windows leave no owned cell
            assert e.code == -7 and ("strips" in names[v] or "tiles" in names[v])
            sim.close()
            continue
        f, g = [t.cpu().numpy() for t in sim.populations()]
        say("variant", names[v])
        if ref is None:
            ref = (f, g)
        else:
            assert np.array_equal(f, ref[0]) and np.array_equal(g, ref[1]), names[v]
        sim.close()
    st = oracle.run(prob, 7)
    assert relmax(ref[0].reshape(st.f.shape), st.f) < TOL[prec]


@pytest.mark.parametrize("prec,tol", [(FP64, 1e-12), (FP32, 1e-5)])
def test_sec5_cases_batch_400_steps(prec, tol):
    """The four MRT cases of Sec. V.B as one batch (4 members of 4 x 800),
    400 steps: every member equals the oracle, and a member run alone is
    bit-identical to the same member in the batch."""
    import paper_1211_3286_amd as rlb
    cases = [wl.qgp_tube_2d(c) for c in "ABCD"]
    sim = rlb.from_problems(cases, precision=prec, diag_every=100)
    say("cases A-D batch prec", prec, "kernel", sim.kernel_name)
    sim.step(400)
    states, sums, bad = gpu_state(sim, cases)
    assert bad == 0
    for c, gs in zip(cases, states):
        st = oracle.run(c, 400)
        F = st.fields()
        err = compare(gs, st, F)
        say("  ", c.name, err)
        assert err["f"] < tol and err["g"] < tol and err["u"] < tol and err["eps"] < tol, err
    one = rlb.from_problems(cases[2], precision=prec)
    one.step(400)
    (g1,), _, _ = gpu_state(one, cases[2])
    assert np.array_equal(g1["g"], states[2]["g"]) and np.array_equal(g1["f"], states[2]["f"])
    s, step, nbad = sim.diagnostics()
    assert step == 400 and nbad == 0


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_periodic_conservation(prec):
    prob = _problem(192, 160, (0, 0, 0))
    sim = gpu_run(prob, 0, prec, diag_every=60)
    s0 = sim.sums()
    sim.step(240)
    s1 = sim.sums()
    d, step, _ = sim.diagnostics()
    drift = np.abs(s1 - s0).max() / np.abs(s0[:2]).max()
    say("d2q9 conservation prec", prec, "drift", drift)
    # FP32: each cell-update rounds its folded-back residual once (unbiased),
    # a random walk of about 1e-8 sqrt(T / cells) relative after T steps
    ncells = prob.params.ncells
    assert drift < (1e-13 if prec == FP64 else 1e-8 * np.sqrt(240 / ncells))
    # the diagnostics of step 240 sum the populations streamed into it
    assert step == 240 and relmax(d, s1) < (1e-13 if prec == FP64 else 1e-10)


def test_fp32_conservation_at_the_bar():
    """The conserved-sum bar of 1e-10 itself, in FP32, on a lattice large
    enough for the rounding random walk (about 1e-8 sqrt(T / cells)) to stay
    below it: 1024 x 1024 for 100 steps, in the variant the autotuner picks."""
    prob = _problem(1024, 1024, (0, 0, 0))
    sim = gpu_run(prob, 0, FP32, diag_every=50)
    res = sim.tune(trial_steps=6)
    s0 = sim.sums()
    sim.step(100)
    s1 = sim.sums()
    drift = np.abs(s1 - s0).max() / np.abs(s0[:2]).max()
    say("d2q9 fp32 conservation 1024^2 x 100,", res["name"], "drift", drift)
    assert drift < 1e-10


def test_host_pointer_populations_and_validation():
    import ctypes
    import torch
    import paper_1211_3286_amd as rlb
    prob = _problem(23, 17, (0, 1, 0))
    sim = gpu_run(prob, 5, FP64)
    f = np.zeros((9, prob.params.ncells))
    g = np.zeros((9, prob.params.ncells))
    assert rlb.lib().rlb_populations(sim.h, f.ctypes.data, g.ctypes.data, 0) == 0
    st = oracle.run(prob, 5)
    assert relmax(f.reshape(st.f.shape), st.f) < 1e-12
    assert relmax(g.reshape(st.g.shape), st.g) < 1e-12
    bad = _problem(23, 17, (0, 1, 0))
    bad.u[2, 0, 3, 4] = 0.01
    with pytest.raises(rlb.RLBError) as ei:
        rlb.from_problems(bad)  # device fields: checked by the validation kernel
    assert ei.value.code == -3
    del torch


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,tol", [(FP32, 1e-5), (FP64, 1e-12)])
def test_full_size_4096_squared_sampled(prec, tol):
    """The 4096 x 4096 periodic benchmark lattice in the autotuned launch
    configuration, sampled cells checked against the oracle on their light
    cones (after K steps a cell depends on its (2K+1)^2 neighbourhood)."""
    import torch
    import paper_1211_3286_amd as rlb
    prob = wl.random_modes(4096, 4096, 1, seed=1211, umax=0.1, amp=0.05, tau_v=0.8,
                           tau_e=0.55, tau_eps=0.7, tau_f=0.8)
    prob.params.lattice = "d2q9"
    K = 4
    sim = rlb.from_problems(prob, precision=prec)
    res = sim.tune(trial_steps=3)
    say("4096^2 d2q9 prec", prec, "tuned", res["name"])
    sim.step(K)
    f, g = sim.populations()
    rng = np.random.default_rng(5)
    cells = [(0, 0, 0), (0, 4095, 4095), (0, 2048, 17)] + [
        (0, int(rng.integers(4096)), int(rng.integers(4096))) for _ in range(5)]
    worst = 0.0
    for c in cells:
        idx = c[1] * 4096 + c[2]
        sub, loc = wl.window(prob, c, K)
        st = oracle.run(sub, K)
        of = st.f[(slice(None),) + loc]
        og = st.g[(slice(None),) + loc]
        scale = max(np.abs(st.f).max(), np.abs(st.g).max())
        err = max(np.abs(f[:, idx].cpu().numpy() - of).max(),
                  np.abs(g[:, idx].cpu().numpy() - og).max()) / scale
        worst = max(worst, err)
    say("  worst sampled error", worst)
    assert worst < tol
    sim.close()
    del f, g
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# Correction term of Eqs. (37)-(38)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("shape", [(131, 129, (0, 1, 0)), (37, 29, (1, 0, 0)), (1, 300, (0, 1, 0)),
                                   (300, 61, (0, 0, 0))],
                         ids=lambda s: f"{s[0]}x{s[1]}_bc{s[2]}")
def test_corrected_step_matches_oracle(prec, shape):
    nx, ny, bc = shape
    prob = _problem(nx, ny, bc)
    prob.params.correction = 1
    T = 25
    sim = gpu_run(prob, T, prec)
    say("d2q9+c7 step", prob.name, "prec", prec, "kernel", sim.kernel_name)
    assert sim.kernel_name.endswith("+c7")
    (gs,), sums, bad = gpu_state(sim, prob)
    st = oracle.run(prob, T)
    F = st.fields()
    err = compare(gs, st, F)
    say("  errors", err)
    assert bad == 0 and st.bad == 0
    assert err["f"] < TOL[prec] and err["g"] < TOL[prec] and err["u"] < TOL[prec], err
    # the correction changes this flow by far more than the GPU-oracle gap
    plain = oracle.run(_problem(nx, ny, bc), T)
    assert relmax(plain.g, st.g) > 100 * max(err["f"], err["g"])


@pytest.mark.parametrize("prec,tol", [(FP64, 1e-11), (FP32, 1e-5)])
def test_corrected_moderate_case_400_steps(prec, tol):
    """The moderately relativistic tube of Sec. V.B (beta up to about 0.55),
    Cases A and D with the correction, as one batch, 400 steps."""
    import paper_1211_3286_amd as rlb
    cases = [wl.qgp_tube_2d(c, a=1.0 / 30.0, moderate=True, correction=True) for c in "AD"]
    sim = rlb.from_problems(cases, precision=prec)
    sim.step(400)
    states, sums, bad = gpu_state(sim, cases)
    assert bad == 0
    for c, gs in zip(cases, states):
        st = oracle.run(c, 400)
        F = st.fields()
        err = compare(gs, st, F)
        say("  ", c.name, "prec", prec, err)
        assert err["f"] < tol and err["g"] < tol and err["u"] < tol and err["eps"] < tol, err


@pytest.mark.parametrize("shape", [(160, 130, (0, 1, 0)), (170, 131, (1, 0, 0)),
                                   (140, 129, (0, 0, 0)), (45, 38, (1, 1, 0))],
                         ids=["lattice", "lattice_ragged_y", "lattice_last_row_alone",
                              "persistent"])
def test_corrected_variants_identical(shape):
    import paper_1211_3286_amd as rlb
    prob = _problem(*shape)
    prob.params.correction = 1
    ref = None
    n = len(rlb.from_problems(prob, precision=FP32).variants())
    for v in range(n):
        sim = rlb.from_problems(prob, precision=FP32)
        sim.variant = v
        try:
            sim.step(6)
        except rlb.RLBError as e:  # rounds whose windows leave no owned cell
            assert e.code == -7 and ("strips" in sim.kernel_name or "tiles" in sim.kernel_name)
            sim.close()
            continue
        g = sim.populations()[1].cpu().numpy()
        if ref is None:
            ref = g
        else:
            assert np.array_equal(g, ref), sim.kernel_name
        sim.close()


# ---------------------------------------------------------------------------
# Strip rounds: narrow members cut into row segments held in LDS, H steps a
# launch (k_d2q9_strips)
# ---------------------------------------------------------------------------
def _strip_members():
    cases = [wl.qgp_tube_2d(c) for c in "AC"]  # 4 x 800, periodic x, zero-gradient y
    more = [_problem(nx, ny, bc, seed=s) for nx, ny, bc, s in
            ((3, 150, (0, 0, 0), 11), (4, 20, (0, 1, 0), 12), (5, 333, (1, 1, 0), 13),
             (1, 97, (0, 0, 0), 14), (7, 1, (0, 0, 0), 15))]
    return cases + more


@pytest.mark.parametrize("corr", [0, 1], ids=["plain", "c7"])
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_strip_rounds_identical_to_one_block_kernel(prec, corr):
    """Every strip-round variant (windows with halos of H or 2H rows, several
    segments per member, partial last rounds, periodic and zero-gradient y,
    widths 1 to 7, a one-row member, a member that fits one window) gives the
    populations of the one-block persistent kernel bit for bit, and the same
    diagnostics sums; the one-block kernel is checked against the oracle."""
    import paper_1211_3286_amd as rlb
    members = _strip_members()
    for m in members:
        m.params.correction = corr
    T = 37
    sim = rlb.from_problems(members, precision=prec, diag_every=10)
    names = sim.variants()
    sim.variant = 0
    sim.step(T)
    ref = [t.cpu().numpy() for t in sim.populations()]
    dref, _, _ = sim.diagnostics()
    states, _, bad = gpu_state(sim, members)
    assert bad == 0
    for p, gs in zip(members, states):
        st = oracle.run(p, T)
        err = compare(gs, st, st.fields())
        assert err["f"] < TOL[prec] and err["g"] < TOL[prec], (p.name, err)
    sim.close()
    ran = 0
    for v, name in enumerate(names):
        if "strips" not in name:
            continue
        s2 = rlb.from_problems(members, precision=prec, diag_every=10)
        s2.variant = v
        s2.step(T)
        f, g = [t.cpu().numpy() for t in s2.populations()]
        d, step, nbad = s2.diagnostics()
        say("strip variant", name, "prec", prec, "corr", corr)
        assert np.array_equal(f, ref[0]) and np.array_equal(g, ref[1]), name
        assert step == T and nbad == 0
        assert relmax(d, dref) < 1e-13, (d, dref)
        ran += 1
        s2.close()
    assert ran == 6


def test_strip_rounds_refuse_wide_members():
    import paper_1211_3286_amd as rlb
    members = _strip_members() + [_problem(200, 5, (0, 1, 0), seed=16)]
    sim = rlb.from_problems(members, precision=FP32)
    for v, name in enumerate(sim.variants()):
        if "strips" in name:
            sim.variant = v
            with pytest.raises(rlb.RLBError) as ei:
                sim.step(2)
            assert ei.value.code == -7
    sim.variant = 0
    sim.step(2)
    assert np.isfinite(sim.sums()).all()


@pytest.mark.parametrize("prec,tol", [(FP64, 1e-12), (FP32, 1e-5)])
def test_sec5_cases_on_strip_rounds_400_steps(prec, tol):
    """The Sec. V.B Cases A-D batch in the autotuned configuration (strip
    rounds win on these 4 x 800 members), 400 steps, against the oracle."""
    import paper_1211_3286_amd as rlb
    cases = [wl.qgp_tube_2d(c) for c in "ABCD"]
    sim = rlb.from_problems(cases, precision=prec)
    res = sim.tune(trial_steps=20)
    say("cases A-D tuned", res["name"])
    sim.step(400)
    states, _, bad = gpu_state(sim, cases)
    assert bad == 0
    for c, gs in zip(cases, states):
        st = oracle.run(c, 400)
        err = compare(gs, st, st.fields())
        say("  ", c.name, err)
        assert err["f"] < tol and err["g"] < tol and err["u"] < tol and err["eps"] < tol, err


# ---------------------------------------------------------------------------
# Tile rounds on the lattice path: windows with halos in LDS, H steps a
# launch (k_d2q9_tiles)
# ---------------------------------------------------------------------------
TILE_SHAPES = [(160, 130, (0, 1, 0)), (45, 700, (1, 0, 0)), (1000, 20, (0, 1, 0)),
               (130, 127, (0, 0, 0)), (4096, 4, (0, 0, 0))]


@pytest.mark.parametrize("corr", [0, 1], ids=["plain", "c7"])
@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("shape", TILE_SHAPES, ids=lambda s: f"{s[0]}x{s[1]}_bc{s[2]}")
def test_tile_rounds_identical_to_one_step_kernel(shape, prec, corr):
    """Every tile-round variant (H = 2 or 3 steps a launch, partial last
    rounds, periodic and zero-gradient faces, an axis shorter than the
    window, 2H halo rows with the correction term) gives the populations and
    the diagnostics sums of the one-step lattice kernel, which the tests
    above check against the oracle; variants whose windows leave no owned
    cell are refused."""
    import paper_1211_3286_amd as rlb
    nx, ny, bc = shape
    prob = _problem(nx, ny, bc, seed=21)
    prob.params.correction = corr
    T = 7
    sim = rlb.from_problems(prob, precision=prec, diag_every=3)
    names = sim.variants()
    assert "lattice" in names[0]
    sim.variant = 0
    sim.step(T)
    ref = [t.cpu().numpy() for t in sim.populations()]
    dref, _, _ = sim.diagnostics()
    sim.close()
    ran = 0
    for v, name in enumerate(names):
        if "tiles" not in name:
            continue
        s2 = rlb.from_problems(prob, precision=prec, diag_every=3)
        s2.variant = v
        try:
            s2.step(T)
        except rlb.RLBError as e:
            # refused: a window that leaves no owned row with the 2H halo of
            # the correction term (64 x 8, and 32 x 16 at H = 4); FP64 with the
            # correction term does not fit a 1024-cell window in LDS
            tx, ty, h = (int(v) for v in re.search(r",(\d+),(\d+)>/h(\d+)", name).groups())
            no_rows = ty - 4 * h < 1
            assert e.code == -7 and corr and (no_rows or (prec == FP64 and tx * ty == 1024)), name
            s2.close()
            continue
        f, g = [t.cpu().numpy() for t in s2.populations()]
        d, step, nbad = s2.diagnostics()
        say("tile variant", name, shape, "prec", prec, "corr", corr)
        assert np.array_equal(f, ref[0]) and np.array_equal(g, ref[1]), name
        assert step == T and nbad == 0
        assert relmax(d, dref) < 1e-13, (name, d, dref)
        ran += 1
        s2.close()
    assert ran >= (1 if corr and prec == FP64 else 5)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_tile_rounds_with_per_cell_taus(prec):
    """Tile rounds with relaxation times from eta/s, against the one-step
    kernel bit for bit and the oracle."""
    import paper_1211_3286_amd as rlb
    prob = _problem(150, 140, (0, 1, 0), seed=22)
    prob.params.eta_s, prob.params.kappa = 0.05, 4 / 3
    prob.params.a_e, prob.params.a_eps = 0.3, 0.6
    T = 11
    sim = rlb.from_problems(prob, precision=prec)
    names = sim.variants()
    sim.variant = 0
    sim.step(T)
    ref = [t.cpu().numpy() for t in sim.populations()]
    (gs,), _, bad = gpu_state(sim, prob)
    st = oracle.run(prob, T)
    err = compare(gs, st, st.fields())
    assert bad == 0 and err["f"] < TOL[prec] and err["g"] < TOL[prec], err
    sim.close()
    for v, name in enumerate(names):
        if "tiles" in name:
            s2 = rlb.from_problems(prob, precision=prec)
            s2.variant = v
            s2.step(T)
            f, g = [t.cpu().numpy() for t in s2.populations()]
            assert np.array_equal(f, ref[0]) and np.array_equal(g, ref[1]), name
            s2.close()


@pytest.mark.parametrize("corr", [0, 1], ids=["plain", "c7"])
@pytest.mark.parametrize("L", [136, 100], ids=["lattice", "persistent"])
def test_inadmissible_cells_counted_like_the_oracle(L, corr):
    """A 2D blast whose outward ring turns cells inadmissible (E <= 0 or
    |M| >= E) within a few steps: every variant of both dispatch paths (one-step
    lattice kernels, tile rounds, per-member and strip rounds), with and
    without the correction term, leaves those cells uncollided and counts them
    like the oracle (FP64 decisions). Next to near-vacuum cells rounding
    differences are amplified, hence the looser population bound."""
    import paper_1211_3286_amd as rlb
    prob = wl.blast_disk(L, correction=corr)
    T = 4
    st = oracle.run(prob, T)
    assert st.bad > 50
    sim = rlb.from_problems(prob, precision=FP64)
    names = sim.variants()
    sim.close()
    ran = 0
    for v, name in enumerate(names):
        sim = rlb.from_problems(prob, precision=FP64)
        sim.variant = v
        try:
            sim.step(T)
        except rlb.RLBError as e:
            # FP64 tile windows of 1024 cells with the correction term do not
            # fit LDS; strip rounds refuse members wider than a strip
            assert e.code == -7 and ((corr and "tiles" in name) or "strips" in name), name
            sim.close()
            continue
        (gs,), _, bad = gpu_state(sim, prob)
        say("  disk", L, "corr", corr, name, "gpu", bad, "oracle", st.bad)
        assert bad == st.bad, name
        assert relmax(gs["f"], st.f) < 1e-10 and relmax(gs["g"], st.g) < 1e-10, name
        ran += 1
        sim.close()
    assert ran >= 2
