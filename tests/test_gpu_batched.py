"""GPU parity of the batched persistent forms.

* Every persistent variant (one block per member, or members cut into
  segments of whole z-planes that wait on their neighbours each step) gives
  bit-identical populations; variant 0 matches the oracle per member.
* A member of a batch evolves bit-identically to the same lattice run alone
  (also when the lone run takes the per-step fused kernel).
* The full sweep: 64 ragged tubes, 3000 steps, one graph launch, FP32, in the
  autotuned configuration; every tube compared with the oracle (two tubes
  with unstable transverse modes at step 1000, see the test).
* The transverse instability of one of those tubes, seeded alike on both
  sides, grows alike.
"""

import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_helpers import gpu_state, relmax, say

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


def _members():
    tubes = wl.tube_batch(n_tubes=5, lmin=300, lmax=900, seed=5)
    cube = wl.random_modes(13, 11, 21, seed=2, umax=0.2, amp=0.1)            # periodic z
    box = wl.random_modes(9, 7, 16, seed=4, umax=0.2, amp=0.1, bc=(1, 1, 1))  # clamped
    return tubes + [cube, box]


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_every_persistent_variant_is_identical(prec):
    import paper_1211_3286_amd as rlb
    members = _members()
    ref = None
    names = rlb.from_problems(members, precision=prec).variants()
    for v, name in enumerate(names):
        sim = rlb.from_problems(members, precision=prec)
        sim.variant = v
        say("persistent variant", v, name, "prec", prec)
        try:
            sim.step(12)
        except rlb.RLBError as e:  # tube rounds need a batch of 1 x 1 x L members
            assert e.code == -7 and "tubes" in name
            continue
        f, g = [t.cpu().numpy() for t in sim.populations()]
        if ref is None:
            ref = (f, g)
            states, _, bad = gpu_state(sim, members)
            assert bad == 0
            for p, gs in zip(members, states):
                st = oracle.run(p, 12)
                tol = 1e-12 if prec == FP64 else 1e-5
                assert relmax(gs["f"], st.f) < tol and relmax(gs["g"], st.g) < tol, p.name
        else:
            assert np.array_equal(f, ref[0]) and np.array_equal(g, ref[1]), name
        sim.close()


def _tubes():
    out = []
    for L, bc, seed in ((1, 1, 1), (5, 1, 2), (100, 1, 3), (300, 1, 4), (700, 1, 5), (1300, 1, 6),
                        (37, 0, 7), (600, 0, 8)):
        t = wl.tube_batch(n_tubes=1, seed=seed, lmin=L, lmax=L)[0]
        t.params.bc = (0, 0, bc)
        out.append(t)
    return out


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_tube_rounds_identical_and_exact(prec):
    """Tube rounds (LDS windows with halos, partial last rounds, periodic and
    zero-gradient ends) against the other persistent kernels and the oracle."""
    import paper_1211_3286_amd as rlb
    tubes = _tubes()
    T = 29  # not a multiple of any round length
    ref = None
    names = rlb.from_problems(tubes, precision=prec).variants()
    oracle_runs = [oracle.run(p, T) for p in tubes]
    want = np.sum([st.fields()["sums"] for st in oracle_runs], axis=0)
    for v, name in enumerate(names):
        sim = rlb.from_problems(tubes, precision=prec, diag_every=1)
        sim.variant = v
        sim.step(T)
        say("tube batch variant", v, name)
        f, g = [t.cpu().numpy() for t in sim.populations()]
        sums, step, bad = sim.diagnostics()
        assert step == T and bad == 0
        assert relmax(sums, want) < (1e-13 if prec == FP64 else 1e-7), name
        if ref is None:
            ref = (f, g)
            off = 0
            for p, st in zip(tubes, oracle_runs):
                nc = p.params.ncells
                tol = 1e-12 if prec == FP64 else 1e-5
                assert relmax(f[:, off:off + nc].reshape(st.f.shape), st.f) < tol, p.name
                assert relmax(g[:, off:off + nc].reshape(st.g.shape), st.g) < tol, p.name
                off += nc
        else:
            assert np.array_equal(f, ref[0]) and np.array_equal(g, ref[1]), name
        # a second call continues from the state (buffer parity across rounds)
        sim.step(3)
        f2 = sim.populations()[0].cpu().numpy()
        if v == 0:
            ref2 = f2
        else:
            assert np.array_equal(f2, ref2), name
        sim.close()


def test_member_equals_single_run():
    import paper_1211_3286_amd as rlb
    tube = wl.tube_batch(n_tubes=1, seed=7)[0]
    cube = wl.random_modes(32, 32, 20, seed=3, umax=0.15)  # alone: per-step fused kernel
    batch = rlb.from_problems([tube, cube], precision=FP32)
    batch.step(40)
    fb, gb = [t.cpu().numpy() for t in batch.populations()]
    off = 0
    for p in (tube, cube):
        one = rlb.from_problems(p, precision=FP32)
        one.step(40)
        say("single run", p.name, one.kernel_name)
        f1, g1 = [t.cpu().numpy() for t in one.populations()]
        nc = p.params.ncells
        assert np.array_equal(fb[:, off:off + nc], f1) and np.array_equal(gb[:, off:off + nc], g1)
        off += nc


def _transverse(g):
    """max |M_x|, |M_y| of a tube's g populations (19 x L), FP64 sums over
    opposite pairs."""
    e = oracle.tables()["e"]
    g = g.reshape(19, -1)
    return max(np.abs(np.asarray(e[:, 0], float) @ g).max(),
               np.abs(np.asarray(e[:, 1], float) @ g).max())


@pytest.mark.timeout(600)
def test_tube_sweep_64x3000():
    """All 64 tubes after 3000 steps, FP32 in the autotuned configuration,
    each against the FP64 oracle. Three of the tubes (6, 29, 46: small tau_v
    with a pressure ratio near 5) have unstable transverse modes: in exact
    arithmetic their mirror-symmetric data keep M_x = M_y = 0, and the GPU's
    pairwise sums keep that symmetry exactly, while the oracle's sequential
    sums leave rounding-level transverse momentum that the instability grows
    to order one after about 1400 steps (then cells turn inadmissible). For
    such a tube the oracle's later state is not a unique result of the
    method: the GPU is compared with it at step 1000, before the growth, and
    must keep the exact symmetry to step 3000 with no inadmissible cell."""
    import paper_1211_3286_amd as rlb
    tubes = wl.tube_batch()
    sim = rlb.from_problems(tubes, precision=FP32, diag_every=1000)
    res = sim.tune(trial_steps=20)
    say("batched tuned", res["name"])
    sim.step(1000)
    early, _, bad1000 = gpu_state(sim, tubes)
    sim.step(2000)
    states, sums, bad = gpu_state(sim, tubes)
    assert bad == 0
    worst, unstable = 0.0, []
    for i in range(64):
        st = oracle.State.init(tubes[i])
        st.step(1000)
        err1000 = max(relmax(early[i]["f"], st.f), relmax(early[i]["g"], st.g))
        st.step(2000)
        F = st.fields()
        scale = np.abs(st.g).max()
        if _transverse(st.g) < 1e-10 * scale:
            err = max(relmax(states[i]["f"], st.f), relmax(states[i]["g"], st.g),
                      relmax(states[i]["n"], F["n"]), relmax(states[i]["eps"], F["eps"]))
            say("  tube", i, tubes[i].name, "FP32 vs oracle after 3000 steps", f"{err:.3e}")
        else:
            unstable.append(i)
            gsym = _transverse(states[i]["g"])
            say("  tube", i, tubes[i].name, "oracle transverse momentum",
                f"{_transverse(st.g):.2e}", "(rounding-seeded instability, oracle inadmissible",
                st.bad, "); GPU vs oracle at step 1000", f"{err1000:.3e}",
                "GPU transverse momentum at 3000", f"{gsym:.1e}")
            assert gsym < 1e-12 * scale
            err = err1000
        worst = max(worst, err)
    say("  worst of the 64 tubes", f"{worst:.3e}", "unstable tubes", unstable)
    assert worst < 1e-5
    assert len(unstable) <= 3


def test_seeded_transverse_instability_matches_oracle():
    """The transverse instability of tube 29 of the batch, seeded on both
    sides by the same u_x, u_y of 1e-9 (far above either side's rounding), is
    reproduced by the GPU (FP64): at step 1300, grown about 7000-fold, the
    transverse momentum profile agrees with the oracle's to 1e-4 of its size.
    The oracle's own rounding-level transverse momentum, grown alike, moves
    its profile by about 1.5e-5 (a perturbation of eps of 1e-13 or 1e-11
    changes it by that much, not more)."""
    import copy
    import paper_1211_3286_amd as rlb
    t = copy.deepcopy(wl.tube_batch()[29])
    L = t.params.nz
    z = np.arange(L)
    t.u[0, :, 0, 0] = 1e-9 * np.sin(2 * np.pi * z / L * 3 + 0.3)
    t.u[1, :, 0, 0] = 1e-9 * np.cos(2 * np.pi * z / L * 5)
    T = 1300
    st = oracle.run(t, T)
    sim = rlb.from_problems(t, precision=FP64)
    sim.step(T)
    (gs,), _, bad = gpu_state(sim, t)
    e = np.asarray(oracle.tables()["e"], float)
    mo = e.T @ st.g.reshape(19, L)
    mg = e.T @ gs["g"].reshape(19, L)
    err = np.abs(mg[:2] - mo[:2]).max() / np.abs(mo[:2]).max()
    say("seeded instability: oracle max|M_x,y|", np.abs(mo[:2]).max(), "GPU",
        np.abs(mg[:2]).max(), "relative difference", err)
    assert np.abs(mo[:2]).max() > 1e-7  # grown well above the seed's 4e-9
    assert err < 1e-4 and bad == st.bad == 0
