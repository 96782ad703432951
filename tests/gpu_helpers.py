"""Shared helpers of the GPU parity tests (HIP path vs the FP64 oracle)."""

from __future__ import annotations

import sys

import numpy as np


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def relmax(a, b) -> float:
    """max|a - b| / max|b| (the max-norm relative error of an array)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def gpu_run(problem, nsteps, precision, **kw):
    import paper_1211_3286_amd as rlb
    sim = rlb.from_problems(problem, precision=precision, **kw)
    if nsteps:
        sim.step(nsteps)
    return sim


def gpu_state(sim, problems):
    """Populations and fields of a handle, reshaped per member like the oracle."""
    f, g = sim.populations()
    m = sim.moments(allow_unphysical=True)
    f = f.cpu().numpy()
    g = g.cpu().numpy()
    q = f.shape[0]  # 19 (D3Q19) or 9 (D2Q9)
    out = []
    if not isinstance(problems, (list, tuple)):
        problems = [problems]
    off = 0
    for p in problems:
        sh = p.params.shape
        nc = p.params.ncells
        sl = slice(off, off + nc)
        out.append({"f": f[:, sl].reshape((q,) + sh), "g": g[:, sl].reshape((q,) + sh),
                    "n": m["n"][sl].cpu().numpy().reshape(sh),
                    "eps": m["eps"][sl].cpu().numpy().reshape(sh),
                    "P": m["P"][sl].cpu().numpy().reshape(sh),
                    "gamma": m["gamma"][sl].cpu().numpy().reshape(sh),
                    "u": m["u"][:, sl].cpu().numpy().reshape((3,) + sh)})
        off += nc
    return out, m["sums"], m["bad"]


def compare(gpu: dict, st, F: dict) -> dict:
    """Max-norm relative errors of populations and fields against the oracle."""
    return {"f": relmax(gpu["f"], st.f), "g": relmax(gpu["g"], st.g),
            "n": relmax(gpu["n"], F["n"]), "eps": relmax(gpu["eps"], F["eps"]),
            "P": relmax(gpu["P"], F["P"]), "gamma": relmax(gpu["gamma"], F["gamma"]),
            "u": float(np.abs(gpu["u"] - F["u"]).max())}


def variants_equal_variant0(problems, precision, kinds, nsteps, tol, refused=lambda name: False):
    """Run variant 0 of ``problems`` for ``nsteps`` steps and check it against
    the oracle within ``tol``; then every variant whose name contains one of
    ``kinds`` must give the same populations bit for bit (or be refused with
    RLB_E_UNSUPPORTED where ``refused(name)``). Returns the names that ran."""
    import oracle
    import paper_1211_3286_amd as rlb
    sim = rlb.from_problems(problems, precision=precision)
    names = sim.variants()
    sim.variant = 0
    sim.step(nsteps)
    ref = [t.cpu().numpy() for t in sim.populations()]
    states, _, bad = gpu_state(sim, problems)
    assert bad == 0
    for p, gs in zip(problems if isinstance(problems, (list, tuple)) else [problems], states):
        st = oracle.run(p, nsteps)
        err = compare(gs, st, st.fields())
        assert err["f"] < tol and err["g"] < tol, (p.name, err)
    sim.close()
    ran = []
    for v, name in enumerate(names):
        if not any(k in name for k in kinds):
            continue
        s2 = rlb.from_problems(problems, precision=precision)
        s2.variant = v
        try:
            s2.step(nsteps)
        except rlb.RLBError as e:
            assert e.code == -7 and refused(name), name
            s2.close()
            continue
        f, g = [t.cpu().numpy() for t in s2.populations()]
        say("  variant", name, "prec", precision)
        assert np.array_equal(f, ref[0]) and np.array_equal(g, ref[1]), name
        ran.append(name)
        s2.close()
    return ran
