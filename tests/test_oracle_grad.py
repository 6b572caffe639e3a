"""Pins of the oracle's variable-projection adjoint: complex-step derivatives of
the forward map (an independent route to the same derivative), central finite
differences, and exact invariants of the cost in the material parameters."""
import numpy as np
import pytest

import workloads as W


def _hn(orc, p, om, jac=False):
    params = np.zeros((1, 16))
    params[0, :5] = p
    return orc.material_eval([W.KIND_HN], params, [0, len(om)], om, jac=jac)


CASES = [
    # (material params, theta, damping, flags)
    ([3.0, 20.0, 1e-9, 0.7, 0.6], [-11.1, -9.7, -8.6, -7.4], 1e-8, 0),
    ([3.0, 20.0, 1e-9, 0.7, 0.6], [-11.1, -9.7, -8.6, -7.4], 1e-8, 1),
    ([5.5, 60.0, 3e-10, 0.4, 0.9], [-11.5, -10.6, -9.9, -9.0, -8.1, -7.2], 1e-8, 0),
    ([2.7, 5.9, 9.4e-10, 0.91, 0.45], [-11.8, -10.0, -9.0, -8.3], 0.0, 0),
    ([4.0, 30.0, 5e-9, 0.8, 0.3], [-11.0, -9.1, -8.8, -7.5, -10.2], 1e-4, 0),
]


@pytest.mark.parametrize("p,th,lam,flags", CASES)
def test_adjoint_matches_complex_step(orc, p, th, lam, flags):
    om = W.log_grid(1e6, 1e10, 180)
    er, ei = _hn(orc, p, om)
    th = np.array(th)
    N = len(th)
    b = orc.Batch([0, len(om)], [0, 1], [N], om, er, ei)
    cost, gt, gr, gi, st = orc.fit_grad(b, th[None], damping=lam, flags=flags)
    assert st[0] == 0
    cs_t, cs_r, cs_i = orc.fit_cs_grad(om, er, ei, th, damping=lam, flags=flags)
    sc = np.max(np.abs(cs_t))
    np.testing.assert_allclose(gt[0], cs_t, rtol=1e-9, atol=1e-10 * sc)
    sr = np.max(np.abs(cs_r))
    np.testing.assert_allclose(gr, cs_r, rtol=1e-9, atol=1e-10 * sr)
    si = np.max(np.abs(cs_i))
    np.testing.assert_allclose(gi, cs_i, rtol=1e-8, atol=1e-10 * si)


def test_adjoint_matches_central_differences(orc):
    om = W.log_grid(1e6, 1e10, 300)
    er, ei = _hn(orc, [3.0, 20.0, 1e-9, 0.7, 0.6], om)
    th = np.array([-11.1, -9.7, -8.6, -7.4, -10.3])
    b = orc.Batch([0, 300], [0, 1], [5], om, er, ei)
    _, gt, _, _, _ = orc.fit_grad(b, th[None])
    st, z, _, _, _ = orc.fit_detail(om, er, ei, th)
    assert np.min(np.abs(z)) >= 1e-3 * np.max(np.abs(z))  # away from flip kinks
    h = 1e-6
    P = 2 * len(th)
    pts = np.repeat(th[None], P, axis=0)
    for i in range(len(th)):
        pts[2 * i, i] += h
        pts[2 * i + 1, i] -= h
    bb = orc.Batch([0, 300], [0, P], [5], om, er, ei)
    c = orc.fit_eval(bb, pts)[0]
    fd = (c[0::2] - c[1::2]) / (2 * h)
    np.testing.assert_allclose(gt[0], fd, rtol=1e-5, atol=1e-6 * np.max(np.abs(fd)))


def test_material_parameter_invariants(orc):
    # d C / d eps_inf(material) = 0 (the fitted eps_inf absorbs it) and
    # d C / d d_eps(material) = 2 C / d_eps (the cost is quadratic in the scale)
    om = W.log_grid(1e5, 1e11, 400)
    p = [3.3, 25.0, 2e-9, 0.75, 0.55]
    er, ei, J = _hn(orc, p, om, jac=True)
    th = np.array([-12.0, -10.8, -9.5, -8.6, -7.3, -6.5])
    b = orc.Batch([0, 400], [0, 1], [6], om, er, ei)
    cost, gt, gr, gi, st = orc.fit_grad(b, th[None])
    g = J[:, :, 0].T @ gr + J[:, :, 1].T @ gi        # chain rule through Eq. 4
    assert abs(g[0]) <= 1e-10 * cost[0]
    assert g[1] == pytest.approx(2 * cost[0] / p[1], rel=1e-9)
    # tau0, alpha, beta against finite differences of the full pipeline
    for q, h in [(2, 1e-6 * p[2]), (3, 1e-6), (4, 1e-6)]:
        pp, pm = list(p), list(p)
        pp[q] += h
        pm[q] -= h
        rp, ip = _hn(orc, pp, om)
        rm, im_ = _hn(orc, pm, om)
        cp = orc.fit_eval(orc.Batch([0, 400], [0, 1], [6], om, rp, ip), th[None])[0][0]
        cm = orc.fit_eval(orc.Batch([0, 400], [0, 1], [6], om, rm, im_), th[None])[0][0]
        assert g[q] == pytest.approx((cp - cm) / (2 * h), rel=1e-5)


def test_grad_cost_weighting_and_target_sum(orc):
    om = W.log_grid(1e6, 1e10, 100)
    er, ei = _hn(orc, [3.0, 20.0, 1e-9, 0.7, 0.6], om)
    th = np.array([[-11.0, -9.5, -8.0], [-10.5, -9.0, -7.5]])
    b = orc.Batch([0, 100], [0, 2], [3], om, er, ei)
    _, g1, r1, i1, _ = orc.fit_grad(b, th)
    _, g2, r2, i2, _ = orc.fit_grad(b, th, grad_cost=np.array([2.0, -0.5]))
    np.testing.assert_allclose(g2[0], 2 * g1[0], rtol=1e-15)
    np.testing.assert_allclose(g2[1], -0.5 * g1[1], rtol=1e-15)
    b1 = orc.Batch([0, 100], [0, 1], [3], om, er, ei)
    _, _, ra, ia, _ = orc.fit_grad(b1, th[:1])
    _, _, rb, ib, _ = orc.fit_grad(b1, th[1:])
    np.testing.assert_allclose(r2, 2 * ra - 0.5 * rb, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(i2, 2 * ia - 0.5 * ib, rtol=1e-12, atol=1e-12)
