"""GPU parity with relaxation times set per cell from eta/s (Sec. III.B):
the D3Q19 and D2Q9 kernels built for it, on both dispatch paths, against the
FP64 oracle, including the paper's shock tubes (the Sec. III.B tube with its
three tau_f choices as one batch, the Sec. V.B Cases A-D at eta/s = 0.5 and
the corrected moderately relativistic case).

Tolerances (max-norm relative): FP64 1e-12 (1e-11 for the 400-step tubes),
FP32 1e-5.
"""

import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_helpers import compare, gpu_run, gpu_state, say, variants_equal_variant0

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
TOL = {FP64: 1e-12, FP32: 1e-5}


def _random(nx, ny, nz, bc, lattice, eta_s=0.1, kappa=1.0):
    p = wl.random_modes(nx, ny, nz, seed=17, umax=0.2, amp=0.1, tau_v=0.8, tau_e=0.6,
                        tau_eps=0.7, tau_f=0.7, bc=bc)
    p.params.lattice = lattice
    p.params.eta_s, p.params.kappa = eta_s, kappa
    p.params.a_e, p.params.a_f = 0.4, 0.8
    return p


def _check(prob, T, prec, tol, **kw):
    sim = gpu_run(prob, T, prec, **kw)
    say("eta/s", prob.name, "prec", prec, "kernel", sim.kernel_name)
    (gs,), sums, bad = gpu_state(sim, prob)
    st = oracle.run(prob, T)
    F = st.fields()
    err = compare(gs, st, F)
    say("  errors", err)
    assert bad == 0 and st.bad == 0
    assert err["f"] < tol and err["g"] < tol and err["u"] < tol and err["eps"] < tol, err
    return sim


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("shape", [(40, 30, 20, (0, 0, 0)), (13, 11, 7, (1, 0, 1))],
                         ids=["lattice", "persistent"])
def test_d3q19_step_matches_oracle(prec, shape):
    _check(_random(*shape, "d3q19"), 25, prec, TOL[prec])


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("shape", [(131, 129, 1, (0, 1, 0)), (37, 29, 1, (1, 0, 0))],
                         ids=["lattice", "persistent"])
def test_d2q9_step_matches_oracle(prec, shape):
    _check(_random(*shape, "d2q9", kappa=4 / 3), 25, prec, TOL[prec])


@pytest.mark.parametrize("prec,tol", [(FP64, 1e-11), (FP32, 1e-5)])
def test_sec3_tube_three_tau_f_batch(prec, tol):
    """Sec. III.B: the 1 x 1 x 800 tube at eta/s = 0.1 with tau_f = tau_g,
    1.0 and 0.6 as one batch, 400 steps, in the autotuned configuration
    (segmented launches are not offered with per-cell relaxation times; the
    autotuner skips them)."""
    import paper_1211_3286_amd as rlb
    tubes = [wl.qgp_tube_3d(0.1, tau_f=tf) for tf in ("tau_g", 1.0, 0.6)]
    sim = rlb.from_problems(tubes, precision=prec)
    res = sim.tune(trial_steps=20)
    say("sec3 batch tuned", res["name"])
    assert "segments" not in res["name"]
    sim.step(400)
    states, sums, bad = gpu_state(sim, tubes)
    assert bad == 0
    for t, gs in zip(tubes, states):
        st = oracle.run(t, 400)
        err = compare(gs, st, st.fields())
        say("  ", t.name, err)
        assert err["f"] < tol and err["g"] < tol and err["n"] < tol and err["u"] < tol, err


@pytest.mark.parametrize("prec,tol", [(FP64, 1e-11), (FP32, 1e-5)])
def test_sec5_cases_eta_s_batch(prec, tol):
    import paper_1211_3286_amd as rlb
    cases = [wl.qgp_tube_2d(c, eta_s=0.5) for c in "ABCD"]
    sim = rlb.from_problems(cases, precision=prec)
    sim.step(400)
    states, sums, bad = gpu_state(sim, cases)
    assert bad == 0
    for c, gs in zip(cases, states):
        st = oracle.run(c, 400)
        err = compare(gs, st, st.fields())
        say("  ", c.name, err)
        assert err["f"] < tol and err["g"] < tol and err["u"] < tol, err


def test_corrected_moderate_case_eta_s():
    """Corrected (Eqs. 37-38) moderately relativistic Case D with per-cell
    relaxation times at eta/s = 0.5, a = 1/30, FP64, 400 steps."""
    prob = wl.qgp_tube_2d("D", a=1.0 / 30.0, moderate=True, correction=True, eta_s=0.5)
    _check(prob, 400, FP64, 1e-11)


@pytest.mark.parametrize("prec,tol", [(FP64, 1e-11), (FP32, 1e-5)])
def test_tube_rounds_with_per_cell_taus(prec, tol):
    """Tube rounds (LDS windows, H steps a launch) with relaxation times from
    eta/s: every round variant equals the one-block persistent kernel bit for
    bit, and the oracle within the tolerance; segmented launches stay refused."""
    import paper_1211_3286_amd as rlb
    tubes = [wl.qgp_tube_3d(0.1, tau_f=0.6, length=L) for L in (300, 500)]
    T = 37
    sim = rlb.from_problems(tubes, precision=prec)
    names = sim.variants()
    sim.variant = 0
    sim.step(T)
    ref = [t.cpu().numpy() for t in sim.populations()]
    states, _, bad = gpu_state(sim, tubes)
    assert bad == 0
    for p, gs in zip(tubes, states):
        st = oracle.run(p, T)
        err = compare(gs, st, st.fields())
        say("  ", p.name, "prec", prec, err)
        assert err["f"] < tol and err["g"] < tol and err["u"] < tol, err
    sim.close()
    checked = 0
    for v, name in enumerate(names):
        if "segments" in name:
            sim = rlb.from_problems(tubes, precision=prec)
            sim.variant = v
            with pytest.raises(rlb.RLBError) as ei:
                sim.step(3)
            assert ei.value.code == -7
            sim.close()
        elif "tubes" in name:
            sim = rlb.from_problems(tubes, precision=prec)
            sim.variant = v
            sim.step(T)
            f, g = [t.cpu().numpy() for t in sim.populations()]
            say("  tube variant", name)
            assert np.array_equal(f, ref[0]) and np.array_equal(g, ref[1]), name
            checked += 1
            sim.close()
    assert checked >= 3


@pytest.mark.parametrize("corr", [0, 1], ids=["plain", "c7"])
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_d2q9_rounds_with_per_cell_taus(prec, corr):
    """Strip rounds (a batch of narrow members), tile rounds and every
    one-step block shape (one lattice) with relaxation times from eta/s, with
    and without the correction term: bit for bit the one-block / first
    one-step kernels, which match the oracle."""
    members = [_random(4, 300, 1, (0, 1, 0), "d2q9", kappa=4 / 3),
               _random(3, 170, 1, (0, 0, 0), "d2q9", kappa=4 / 3)]
    for m in members:
        m.params.correction = corr
    ran = variants_equal_variant0(members, prec, ("strips",), 13, TOL[prec])
    assert len(ran) == 6
    lat = _random(150, 130, 1, (0, 1, 0), "d2q9", kappa=4 / 3)
    lat.params.correction = corr
    big = lambda n: ",32,32>" in n or ",64,16>" in n
    ran = variants_equal_variant0(
        [lat], prec, ("tiles", "k_d2q9_lattice"), 13, TOL[prec],
        refused=lambda n: corr and (",64,8>" in n or (prec == FP64 and big(n))))
    assert len(ran) >= (1 if corr and prec == FP64 else 5)
