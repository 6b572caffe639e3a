"""Automatic pole count and the average fractional error on the GPU against
the oracle: the error of given expansions, and the whole search (fitted in
chunks of pole counts on the GPU, one pole count at a time in the oracle)."""
import numpy as np
import pytest

import workloads as W
from _helpers import small_ragged, targets_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    import paper_2109_01928_amd as D

    assert torch.cuda.is_available()
    D.lib()
    return D


def _t(x):
    import torch
    return torch.tensor(x, device="cuda")


def test_afe_matches_oracle(D, orc):
    import torch
    wl = small_ragged(10, seed=41, Fr=(20, 400), Nr=(1, 24), Pr=(1, 6))
    er, ei = targets_oracle(orc, wl)
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=6)
    ob = orc.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, er, ei)
    c, w, e, st = orc.fit_eval(ob, theta)
    b = D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, _t(er), _t(ei))
    g = D.afe(b, _t(theta), _t(np.nan_to_num(w)), _t(e)).cpu().numpy()
    for cI in range(wl.P):
        m = int(np.searchsorted(wl.cand_off, cI, side="right") - 1)
        a, z, n = wl.f_off[m], wl.f_off[m + 1], wl.n_poles[m]
        ref = orc.afe(wl.omega[a:z], er[a:z], ei[a:z], w[cI, :n], 10.0 ** theta[cI, :n], e[cI])
        assert g[cI] == pytest.approx(ref, rel=1e-12), cI


def test_fit_auto_matches_oracle(D, orc):
    om = W.log_grid(1e6, 1e10, 120)
    x1 = om * 1e-9
    er1, ei1 = 4.0 + 20.0 / (1 + x1 * x1), 20.0 * x1 / (1 + x1 * x1)
    wl = W.hn_cc(M=3, F=120, N=1, P=1, iters=0, seed=5)
    er3, ei3 = orc.material_eval(wl.kind, wl.params, wl.f_off, wl.omega)
    x2a, x2b = om * 2e-11, om * 3e-8
    er2 = 3.0 + 12.0 / (1 + x2a * x2a) + 30.0 / (1 + x2b * x2b)
    ei2 = 12.0 * x2a / (1 + x2a * x2a) + 30.0 * x2b / (1 + x2b * x2b)
    f_off = np.array([0, 120, 240, 360, 480, 600])
    omega = np.concatenate([om, wl.omega, om])
    er = np.concatenate([er1, er3, er2])
    ei = np.concatenate([ei1, ei3, ei2])
    lb, ub = np.full(5, -12.0), np.full(5, -6.0)
    kw = dict(n_max=7, afe_target=5.0, particles=24, iters=30, seed=3, polish_steps=10)
    on, oth, ow, oe, oa = orc.fit_auto(f_off, omega, er, ei, lb, ub, **kw)
    b = D.Batch(f_off, np.arange(6), np.ones(5, np.int32), omega, _t(er), _t(ei))
    gn, gth, gw, ge, ga = (t.cpu().numpy() for t in D.fit_auto(b, _t(lb), _t(ub), chunk=3, **kw))
    print("pole counts: GPU", gn, "oracle", on, "AFE GPU", ga, "oracle", oa)
    np.testing.assert_array_equal(gn, on)
    np.testing.assert_allclose(ga, oa, rtol=1e-4)
    assert on[0] == 1 and on[4] <= 2
    for m in range(5):
        n = on[m]
        np.testing.assert_allclose(gth[m, :n], oth[m, :n], rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(gw[m, :n], ow[m, :n], rtol=1e-4, atol=1e-6 * np.max(np.abs(ow[m, :n])))
        assert np.all(np.isnan(gth[m, n:]))
