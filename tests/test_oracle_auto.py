"""Pins of the oracle's automatic pole count (Sec. III-B: poles are added
from one until the average fractional error is below 5 % or 20 poles): an
exact single-pole material stops at one pole with a vanishing error, an exact
three-pole material never needs more than three, the error target is met
whenever the search stops early, and a larger target never needs more poles."""
import numpy as np

import workloads as W


def _debye_sum(orc, om, einf, pairs):
    # eps = einf + sum d / (1 + j w tau) with the loss sign of Eq. 1, written out
    er = np.full(len(om), einf, dtype=np.float64)
    ei = np.zeros(len(om))
    for d, tau in pairs:
        x = om * tau
        er += d / (1 + x * x)
        ei += d * x / (1 + x * x)
    return er, ei


def test_exact_debye_materials(orc):
    om = W.log_grid(1e6, 1e10, 120)
    er1, ei1 = _debye_sum(orc, om, 4.0, [(20.0, 1e-9)])
    er3, ei3 = _debye_sum(orc, om, 3.0, [(10.0, 3e-11), (25.0, 1e-9), (15.0, 4e-8)])
    f_off = [0, 120, 240]
    omega = np.concatenate([om, om])
    n, th, w, einf, err = orc.fit_auto(f_off, omega, np.concatenate([er1, er3]), np.concatenate([ei1, ei3]),
                                       -12.0, -6.0, n_max=6, particles=24, iters=40, seed=1)
    assert n[0] == 1 and err[0] < 1e-3
    np.testing.assert_allclose(10.0 ** th[0, 0], 1e-9, rtol=1e-4)
    np.testing.assert_allclose(w[0, 0], 20.0, rtol=1e-4)
    assert 1 <= n[1] <= 3 and err[1] < 5.0
    assert np.all(np.isnan(th[0, 1:])) and np.all(np.isnan(th[1, n[1]:]))


def test_target_met_or_maximum_reached_and_monotone_in_target(orc):
    wl = W.hn_cc(M=3, F=150, N=1, P=1, iters=0, seed=5)
    er, ei = orc.material_eval(wl.kind, wl.params, wl.f_off, wl.omega)
    kw = dict(n_max=8, particles=24, iters=30, seed=2, polish_steps=10)
    n5, _, _, _, e5 = orc.fit_auto(wl.f_off, wl.omega, er, ei, wl.lb, wl.ub, afe_target=5.0, **kw)
    n20, _, _, _, e20 = orc.fit_auto(wl.f_off, wl.omega, er, ei, wl.lb, wl.ub, afe_target=20.0, **kw)
    for n, e, target in ((n5, e5, 5.0), (n20, e20, 20.0)):
        assert np.all((e < target) | (n == 8))
    assert np.all(n20 <= n5)
