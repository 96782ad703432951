"""GPU parity of the batched persistent forms.

* Every persistent variant (one block per member, or members cut into
  segments of whole z-planes that wait on their neighbours each step) gives
  bit-identical populations; variant 0 matches the oracle per member.
* A member of a batch evolves bit-identically to the same lattice run alone
  (also when the lone run takes the per-step fused kernel).
* The full sweep: 64 ragged tubes, 3000 steps, one graph launch, FP32, in the
  autotuned configuration; a subset of tubes compared with the oracle.
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


@pytest.mark.timeout(600)
def test_tube_sweep_64x3000():
    import paper_1211_3286_amd as rlb
    tubes = wl.tube_batch()
    sim = rlb.from_problems(tubes, precision=FP32, diag_every=1000)
    res = sim.tune(trial_steps=20)
    say("batched tuned", res["name"])
    sim.step(3000)
    states, sums, bad = gpu_state(sim, tubes)
    assert bad == 0
    worst = 0.0
    for i in range(0, 64, 8):
        st = oracle.run(tubes[i], 3000)
        err = max(relmax(states[i]["f"], st.f), relmax(states[i]["g"], st.g))
        say("  tube", i, tubes[i].name, "FP32 vs oracle", err)
        worst = max(worst, err)
    assert worst < 1e-5
