"""Pins of the oracle against the qualitative findings the paper reports for
its shock-tube experiments (its figures and the transport-model data they
compare with are not available; the text states what they show).

* Sec. III.B, Fig. 1 (E1): at t = 400 the particle-number profile of
  tau_f = tau_g departs more and more from those of tau_f = 1.0 and 0.6 as
  eta/s grows over 0.01, 0.05, 0.1, and gets smoother.
* Sec. V.B, Fig. 3 (E3): in Case D the discontinuity at the membrane fades
  as a decreases over 1, 1/5, 1/20, 1/50; a = 1/20 and 1/50 differ little.
* Sec. V.B, Figs. 4-5 (E4): Cases A and B (no visible difference between
  them) show a pressure discontinuity at the membrane that grows from
  eta/s = 0.2 to 0.5; Case D shows none.
(E2, the velocity jumps of Cases A-D, and E5, beta of about 0.55 in the
moderately relativistic tube, are pinned with the relaxation-time tests.)

The discontinuity of a profile x is the step across the membrane (cells 399
and 400) in excess of the larger neighbouring step, over max |x|.
"""

import numpy as np
import pytest

import workloads as wl


def _excess(x):
    return (abs(x[400] - x[399]) - max(abs(x[399] - x[398]), abs(x[401] - x[400]))) / np.abs(x).max()


def test_e1_tau_f_dependence_grows_with_eta_s(orc):
    d1, d2, smooth = [], [], []
    for es in (0.01, 0.05, 0.1):
        n = {tf: orc.run(wl.qgp_tube_3d(es, tau_f=tf), 400).fields()["n"].ravel()
             for tf in ("tau_g", 1.0, 0.6)}
        d1.append(np.abs(n["tau_g"] - n[1.0]).max() / np.abs(n[1.0]).max())
        d2.append(np.abs(n["tau_g"] - n[0.6]).max() / np.abs(n[0.6]).max())
        smooth.append(np.abs(np.diff(n["tau_g"])).max())
    assert d1[0] < d1[1] < d1[2] and d2[0] < d2[1] < d2[2], (d1, d2)
    assert smooth[0] > smooth[1] > smooth[2], smooth


def test_e3_case_d_discontinuity_fades_with_a(orc):
    u = {a: orc.run(wl.qgp_tube_2d("D", a=a, eta_s=0.5), 400).fields()["u"][1, 0, :, 0]
         for a in (1.0, 1 / 5, 1 / 20, 1 / 50)}
    ex = [_excess(u[a]) for a in (1.0, 1 / 5, 1 / 20, 1 / 50)]
    assert ex[0] > ex[1] > ex[2] > ex[3], ex
    assert ex[0] > 0.01 and ex[2] < 1e-3, ex
    # a = 1/20 suffices: going on to 1/50 changes the profile several times
    # less than going from 1 to 1/20
    assert np.abs(u[1 / 20] - u[1 / 50]).max() < 0.25 * np.abs(u[1.0] - u[1 / 20]).max()


def test_e4_pressure_discontinuity_grows_with_eta_s(orc):
    ex = {}
    for es in (0.2, 0.5):
        P = {c: orc.run(wl.qgp_tube_2d(c, eta_s=es), 400).fields()["P"][0, :, 0] for c in "ABD"}
        assert np.abs(P["A"] - P["B"]).max() < 1e-6 * np.abs(P["A"]).max()  # tau_q: no effect
        ex[es] = {c: _excess(P[c]) for c in "AD"}
    assert ex[0.5]["A"] > 2 * ex[0.2]["A"] > 0, ex
    assert ex[0.2]["D"] < 0.1 * ex[0.2]["A"] and ex[0.5]["D"] < 0.1 * ex[0.5]["A"], ex
