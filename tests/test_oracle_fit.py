"""Pins of the oracle's cost evaluation (Eq. 7 basis, damped LS weights on the
loss part, sign flip, eps_inf, real+imaginary cost; Sec. III-B) against the
paper's printed worked example, exact rational arithmetic, closed forms,
library routines, brute force and invariants."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _batch(orc, omega, er, ei, N, P=1):
    F = len(omega)
    return orc.Batch([0, F], [0, P], [N], omega, er, ei)


def _hn_target(orc, p, omega):
    params = np.zeros((1, 16))
    params[0, :5] = p
    return orc.material_eval([W.KIND_HN], params, [0, len(omega)], omega)


def _multidebye(omega, einf, de, tau):
    eps = einf + sum(d / (1 + 1j * omega * t) for d, t in zip(de, tau))
    return eps.real.copy(), -eps.imag.copy()


@pytest.mark.parametrize("damping", [0.0, 1e-8, 1e-6])
def test_listing2_worked_example(orc, damping):
    g = json.load(open(os.path.join(GOLD, "listing2.json")))
    m = g["material"]
    F = 100
    om = W.log_grid(g["band_hz"][0], g["band_hz"][1], F)
    er, ei = _hn_target(orc, [m["eps_inf"], m["d_eps"], m["tau0"], m["alpha"], m["beta"]], om)
    th = np.log10(np.array(g["printed_tau"]))[None, :]
    cost, w, einf, st = orc.fit_eval(_batch(orc, om, er, ei, 5), th, damping=damping)
    assert st[0] == 0
    np.testing.assert_array_equal(np.round(w[0], 4), g["printed_d_eps"])
    assert round(float(einf[0]), 4) == g["printed_eps_inf"]


def test_listing2_rejects_other_readings(orc):
    # The printed digits single out F = 100 and the loss-only LS: F = 50 / 200
    # give different 4-decimal weights.
    g = json.load(open(os.path.join(GOLD, "listing2.json")))
    m = g["material"]
    th = np.log10(np.array(g["printed_tau"]))[None, :]
    for F in (50, 200):
        om = W.log_grid(1e7, 1e11, F)
        er, ei = _hn_target(orc, [m["eps_inf"], m["d_eps"], m["tau0"], m["alpha"], m["beta"]], om)
        _, w, einf, _ = orc.fit_eval(_batch(orc, om, er, ei, 5), th)
        assert not (np.array_equal(np.round(w[0], 4), g["printed_d_eps"]) and
                    round(float(einf[0]), 4) == g["printed_eps_inf"])


def test_exact_rational_tiny_case(orc):
    # F = 2, N = 1 with w*tau = 1 and 3: R = (1/2, 1/10), I = (1/2, 3/10).
    # Everything below is exact rational arithmetic, independent of the oracle.
    tau = 1e-9
    om = np.array([1.0, 3.0]) / tau
    er = np.array([5.0, 3.0])
    ei = np.array([1.0, 0.0])
    R = [Fraction(1, 2), Fraction(1, 10)]
    I = [Fraction(1, 2), Fraction(3, 10)]
    z = (I[0] * 1 + I[1] * 0) / (I[0] ** 2 + I[1] ** 2)       # = 25/17
    einf = ((5 - z * R[0]) + (3 - z * R[1])) / 2
    rr = [Fraction(5) - einf - z * R[0], Fraction(3) - einf - z * R[1]]
    ri = [Fraction(1) - z * I[0], Fraction(0) - z * I[1]]
    C = sum(a * a for a in rr) + sum(b * b for b in ri)
    cost, w, e, st = orc.fit_eval(_batch(orc, om, er, ei, 1), np.array([[-9.0]]), damping=0.0)
    assert st[0] == 0
    assert w[0, 0] == pytest.approx(float(z), rel=1e-14)
    assert e[0] == pytest.approx(float(einf), rel=1e-14)
    assert cost[0] == pytest.approx(float(C), rel=1e-13)


def test_exact_rational_two_poles(orc):
    # F = 3, N = 2: normal equations solved exactly with Fractions; x = w tau
    # chosen so that every basis value is rational.
    t1, t2 = 1e-9, 2e-9                       # tau2 = 2 tau1
    xs1 = [Fraction(1, 2), Fraction(1), Fraction(2)]
    om = np.array([float(x) for x in xs1]) / t1
    er = np.array([9.0, 7.0, 4.0])
    ei = np.array([2.0, 3.0, 1.0])

    def RI(x):
        return 1 / (1 + x * x), x / (1 + x * x)

    B1 = [RI(x) for x in xs1]
    B2 = [RI(2 * x) for x in xs1]
    I1 = [b[1] for b in B1]
    I2 = [b[1] for b in B2]
    g11 = sum(a * a for a in I1)
    g12 = sum(a * b for a, b in zip(I1, I2))
    g22 = sum(b * b for b in I2)
    b1 = sum(a * Fraction(e) for a, e in zip(I1, [2, 3, 1]))
    b2 = sum(a * Fraction(e) for a, e in zip(I2, [2, 3, 1]))
    det = g11 * g22 - g12 * g12
    z1 = (g22 * b1 - g12 * b2) / det
    z2 = (g11 * b2 - g12 * b1) / det
    w1, w2 = abs(z1), abs(z2)
    mis = [Fraction(e) - w1 * B1[k][0] - w2 * B2[k][0] for k, e in enumerate([9, 7, 4])]
    einf = sum(mis) / 3
    C = sum((m - einf) ** 2 for m in mis) + sum((Fraction(e) - w1 * I1[k] - w2 * I2[k]) ** 2
                                                for k, e in enumerate([2, 3, 1]))
    th = np.log10(np.array([[t1, t2]]))
    cost, w, e, st = orc.fit_eval(_batch(orc, om, er, ei, 2), th, damping=0.0)
    assert st[0] == 0
    np.testing.assert_allclose(w[0], [float(w1), float(w2)], rtol=1e-12)
    assert e[0] == pytest.approx(float(einf), rel=1e-13)
    assert cost[0] == pytest.approx(float(C), rel=1e-11)
    # the same case without the flip keeps the signed weights
    _, wn, _, _ = orc.fit_eval(_batch(orc, om, er, ei, 2), th, damping=0.0, flags=1)
    np.testing.assert_allclose(wn[0], [float(z1), float(z2)], rtol=1e-12)


@pytest.mark.parametrize("damping", [0.0, 1e-8, 1e-3])
def test_single_pole_closed_form(orc, damping):
    # N = 1: the damped normal equation is scalar, z = b / ((1 + damping) G)
    om = W.log_grid(1e6, 1e10, 300)
    er, ei = _hn_target(orc, [3.0, 20.0, 1e-9, 0.7, 0.6], om)
    th = np.array([[-9.3]])
    x = om * 10 ** -9.3
    I = x / (1 + x * x)
    R = 1 / (1 + x * x)
    z = (I @ ei) / ((1 + damping) * (I @ I))
    cost, w, e, st = orc.fit_eval(_batch(orc, om, er, ei, 1), th, damping=damping)
    assert w[0, 0] == pytest.approx(abs(z), rel=1e-12)
    einf = np.mean(er - z * R)
    assert e[0] == pytest.approx(einf, rel=1e-12)
    C = np.sum((er - einf - z * R) ** 2) + np.sum((ei - z * I) ** 2)
    assert cost[0] == pytest.approx(C, rel=1e-11)


def test_exact_recovery_of_true_poles(orc):
    om = W.log_grid(1e6, 1e10, 400)
    tau = np.array([3e-11, 4e-10, 6e-9, 8e-8])
    de = np.array([4.0, 12.0, 7.5, 20.0])
    er, ei = _multidebye(om, 3.25, de, tau)
    cost, w, e, st = orc.fit_eval(_batch(orc, om, er, ei, 4), np.log10(tau)[None], damping=0.0)
    assert st[0] == 0
    np.testing.assert_allclose(w[0], de, rtol=1e-10)
    assert e[0] == pytest.approx(3.25, rel=1e-12)
    assert cost[0] <= 1e-24 * (er @ er + ei @ ei)


def test_normal_equation_identities(orc):
    om = W.log_grid(1e6, 1e10, 500)
    er, ei = _hn_target(orc, [2.5, 33.0, 1e-9, 0.6, 0.7], om)
    th = np.array([-11.0, -10.1, -9.0, -8.2, -7.3])
    R, I = orc.basis(om, th)
    # undamped, no flip: residual orthogonal to the loss basis; real residual has zero mean
    st, z, d, rr, ri = orc.fit_detail(om, er, ei, th, damping=0.0, flags=1)
    assert st == 0
    assert np.max(np.abs(I @ ri)) <= 1e-10 * np.linalg.norm(I) * np.linalg.norm(ei)
    assert abs(rr.sum()) <= 1e-12 * np.abs(er).sum()
    # damped: I^T (eps'' - I z) = damping diag(I^T I) z   (Marquardt scaling)
    lam = 1e-4
    st, z, d, rr, ri = orc.fit_detail(om, er, ei, th, damping=lam, flags=1)
    lhs = I @ (ei - I.T @ z)
    rhs = lam * np.sum(I * I, axis=1) * z
    np.testing.assert_allclose(lhs, rhs, rtol=1e-7, atol=1e-12 * np.abs(rhs).max())
    np.testing.assert_allclose(d, np.linalg.norm(I, axis=1), rtol=1e-14)


@pytest.mark.parametrize("damping", [0.0, 1e-8, 1e-4])
def test_matches_scipy_lstsq_on_stacked_system(orc, damping):
    om = W.log_grid(1e6, 1e10, 256)
    er, ei = _hn_target(orc, [5.0, 50.0, 3e-9, 0.8, 0.5], om)
    th = np.array([-11.5, -10.0, -8.9, -7.6])
    _, I = orc.basis(om, th)
    d = np.linalg.norm(I, axis=1)
    A = np.vstack([(I / d[:, None]).T, math.sqrt(damping) * np.eye(4)])
    y = np.concatenate([ei, np.zeros(4)])
    zt = scipy.linalg.lstsq(A, y, lapack_driver="gelsd")[0]
    st, z, _, _, _ = orc.fit_detail(om, er, ei, th, damping=damping, flags=1)
    assert np.linalg.cond(A) < 1e6
    np.testing.assert_allclose(z, zt / d, rtol=1e-11)


def test_bruteforce_weight_scan(orc):
    # N = 1: the LS weight is the minimiser of sum (eps'' - w I)^2 over w; a
    # fine scan finds it.  N = 2: same on a 2-D grid.
    om = W.log_grid(1e6, 1e10, 120)
    er, ei = _hn_target(orc, [3.0, 20.0, 1e-9, 0.7, 0.6], om)
    for th in (np.array([-9.0]), np.array([-9.8, -8.4])):
        st, z, _, _, _ = orc.fit_detail(om, er, ei, th, damping=0.0, flags=1)
        _, I = orc.basis(om, th)
        if len(th) == 1:
            ws = np.linspace(0, 2 * abs(z[0]) + 1, 200001)
            res = ((ei[None, :] - ws[:, None] * I[0][None, :]) ** 2).sum(1)
            best = ws[np.argmin(res)]
            assert abs(best - z[0]) <= ws[1] - ws[0]
        else:
            g1 = np.linspace(z[0] - 2, z[0] + 2, 801)
            g2 = np.linspace(z[1] - 2, z[1] + 2, 801)
            W1, W2 = np.meshgrid(g1, g2, indexing="ij")
            r = ei[None, None, :] - W1[..., None] * I[0] - W2[..., None] * I[1]
            res = (r * r).sum(-1)
            i, j = np.unravel_index(np.argmin(res), res.shape)
            assert abs(g1[i] - z[0]) <= g1[1] - g1[0] and abs(g2[j] - z[1]) <= g2[1] - g2[0]


def test_bruteforce_tau_grid_single_pole(orc):
    # N = 1 global minimum over log10 tau on a 1e-4 grid: the cost is smooth and
    # the grid minimum brackets a stationary point.
    om = W.log_grid(1e6, 1e10, 200)
    er, ei = _hn_target(orc, [3.0, 20.0, 1e-9, 0.8, 0.7], om)
    grid = np.arange(-12, -7, 1e-4)
    b = orc.Batch([0, 200], [0, len(grid)], [1], om, er, ei)
    cost, _, _, _ = orc.fit_eval(b, grid[:, None])
    k = int(np.argmin(cost))
    assert 0 < k < len(grid) - 1
    assert cost[k] <= cost[k - 1] and cost[k] <= cost[k + 1]
    assert -9.5 < grid[k] < -8.5


def test_invariants(orc):
    om = W.log_grid(1e6, 1e10, 333)
    er, ei = _hn_target(orc, [4.0, 25.0, 2e-9, 0.65, 0.55], om)
    th = np.array([-11.2, -9.9, -8.7, -7.7, -10.4])
    b = _batch(orc, om, er, ei, 5)
    c0, w0, e0, _ = orc.fit_eval(b, th[None])
    # permutation symmetry
    perm = np.array([3, 0, 4, 1, 2])
    c1, w1, e1, _ = orc.fit_eval(b, th[perm][None])
    assert c1[0] == pytest.approx(c0[0], rel=1e-12)
    np.testing.assert_allclose(w1[0], w0[0][perm], rtol=1e-10)
    # scaling the whole target scales the cost quadratically (damping is scale free)
    s = 3.7
    c2, w2, e2, _ = orc.fit_eval(_batch(orc, om, s * er, s * ei, 5), th[None])
    assert c2[0] == pytest.approx(s * s * c0[0], rel=1e-12)
    np.testing.assert_allclose(w2[0], s * w0[0], rtol=1e-10)
    # shifting eps' by a constant only moves eps_inf
    c3, w3, e3, _ = orc.fit_eval(_batch(orc, om, er + 1.5, ei, 5), th[None])
    assert c3[0] == pytest.approx(c0[0], rel=1e-11)
    assert e3[0] == pytest.approx(e0[0] + 1.5, rel=1e-13)


def test_sign_flip_penalises_negative_weights(orc):
    # target built with one negative Debye weight: without the flip the fit is
    # exact; with the flip (Sec. III-B) the weight turns positive and the cost
    # becomes the misfit of the flipped model
    om = W.log_grid(1e6, 1e10, 300)
    tau = np.array([1e-9, 5e-11])
    er, ei = _multidebye(om, 3.0, [10.0, -2.0], tau)
    th = np.log10(tau)[None]
    b = _batch(orc, om, er, ei, 2)
    cn, wn, en, _ = orc.fit_eval(b, th, damping=0.0, flags=1)
    assert cn[0] < 1e-20
    np.testing.assert_allclose(wn[0], [10.0, -2.0], rtol=1e-10)
    cf, wf, ef, _ = orc.fit_eval(b, th, damping=0.0)
    np.testing.assert_allclose(wf[0], [10.0, 2.0], rtol=1e-10)
    # flipped model misses by 4 x the second pole (real part up to its mean)
    mr, mi = _multidebye(om, 0.0, [4.0], tau[1:])
    expect = np.sum((mr - mr.mean()) ** 2) + np.sum(mi ** 2)
    assert cf[0] == pytest.approx(expect, rel=1e-9)


def test_status_codes(orc):
    om = W.log_grid(1e6, 1e10, 50)
    er, ei = _hn_target(orc, [3.0, 20.0, 1e-9, 0.7, 0.6], om)
    b = orc.Batch([0, 50], [0, 4], [3], om, er, ei)
    th = np.array([[-9, -8, -10], [-9, -9, -10], [np.nan, -8, -10], [-9, -8, 70.0]])
    c, w, e, st = orc.fit_eval(b, th, damping=0.0)
    assert list(st) == [0, 2, 1, 1]
    assert np.isfinite(c[0]) and c[1] == np.inf and np.isnan(c[2]) and np.isnan(c[3])
    # with damping, duplicate relaxation times are solvable (equal split)
    b2 = orc.Batch([0, 50], [0, 2], [3], om, er, ei)
    c, w, e, st = orc.fit_eval(b2, th[:2], damping=1e-8)
    assert list(st) == [0, 0]
    assert w[1, 0] == pytest.approx(w[1, 1], rel=1e-6)
    # non-finite targets
    ei2 = ei.copy()
    ei2[7] = np.inf
    c, w, e, st = orc.fit_eval(orc.Batch([0, 50], [0, 1], [3], om, er, ei2), th[:1])
    assert st[0] == 1 and np.isnan(c[0])


def test_long_double_agrees(orc):
    wl = W.mixed_uniform(M=4, F=200, N=6, P=16, iters=1, seed=3)
    er, ei = orc.material_eval(wl.kind, wl.params, wl.f_off, wl.omega)
    b = orc.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, er, ei)
    th = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, 1)
    c64, w64, _, _ = orc.fit_eval(b, th)
    c80, w80, _, _ = orc.fit_eval(b, th, precision=80)
    np.testing.assert_allclose(c64, c80, rtol=1e-8)


def test_afe_metric(orc):
    om = W.log_grid(1e6, 1e10, 100)
    de = np.array([3.0, 5.0])
    tau = np.array([1e-9, 1e-10])
    er, ei = _multidebye(om, 2.0, de, tau)
    assert orc.afe(om, er, ei, de, tau, 2.0) == pytest.approx(0.0, abs=1e-12)
    # a model that is uniformly (1+d) x the data misses by d in each part
    d = 0.02
    assert orc.afe(om, er * (1 + d), ei * (1 + d), de, tau, 2.0) == pytest.approx(
        100 * 2 * d / (1 + d), rel=1e-10)
