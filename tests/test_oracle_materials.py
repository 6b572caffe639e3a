"""Pins of the oracle's material models (Eqs. 1, 3-6) against closed forms,
printed values and invariants that do not come from the oracle itself."""
import math

import numpy as np
import pytest

import workloads as W


def _one(orc, kind, p, omega, noise_seed=0, jac=False):
    params = np.zeros((1, 16))
    params[0, :len(p)] = p
    return orc.material_eval([kind], params, [0, len(omega)], omega, noise_seed=noise_seed, jac=jac)


def test_fig1_single_debye_values(orc):
    # Fig. 1 caption: eps_s = 15, eps_inf = 1, tau0 = 0.1 ns, f0 = 1/(2 pi tau0).
    # At f0 the real part is halfway (eps_s+eps_inf)/2 = 8 and the loss peaks at
    # (eps_s-eps_inf)/2 = 7 (Eq. 3).
    tau0 = 1e-10
    f0 = 1 / (2 * math.pi * tau0)
    assert abs(f0 - 1.5915494309e9) < 1.0
    om = np.array([2 * math.pi * f0])
    for kind, p in [(W.KIND_DEBYE, [1.0, 14.0, tau0]), (W.KIND_HN, [1.0, 14.0, tau0, 1.0, 1.0])]:
        er, ei = _one(orc, kind, p, om)
        assert er[0] == pytest.approx(8.0, rel=1e-15)
        assert ei[0] == pytest.approx(7.0, rel=1e-15)
    # the loss is largest at f0 (relaxation frequency definition below Eq. 3)
    om = 2 * math.pi * np.logspace(8, 11, 3001)
    er, ei = _one(orc, W.KIND_DEBYE, [1.0, 14.0, tau0], om)
    k = int(np.argmax(ei))
    assert abs(om[k] / (2 * math.pi) / f0 - 1) < 3e-3
    # the real part is decreasing (eps' goes from eps_s to eps_inf)
    assert np.all(np.diff(er) < 0)
    er, ei = _one(orc, W.KIND_DEBYE, [1.0, 14.0, tau0], 2 * math.pi * np.array([1e3, 1e17]))
    assert er[0] == pytest.approx(15.0, rel=1e-12) and er[1] == pytest.approx(1.0, rel=1e-12)


def _cole_cole_textbook(w, einf, de, tau, a):
    # Cole & Cole (1941) real/imaginary parts for eps_inf + de/(1+(j w tau)^a)
    y = (w * tau) ** a
    c, s = math.cos(a * math.pi / 2), math.sin(a * math.pi / 2)
    den = 1 + 2 * y * c + y * y
    return einf + de * (1 + y * c) / den, de * y * s / den


def _cole_davidson_textbook(w, einf, de, tau, b):
    # Davidson & Cole (1951): eps_inf + de cos^b(phi) e^{-j b phi}, phi = atan(w tau)
    phi = math.atan(w * tau)
    amp = de * math.cos(phi) ** b
    return einf + amp * math.cos(b * phi), amp * math.sin(b * phi)


@pytest.mark.parametrize("a", [0.3, 0.55, 0.91, 1.0])
def test_hn_reduces_to_cole_cole(orc, a):
    om = W.log_grid(1e5, 1e11, 257)
    p = [2.7, 5.9, 9.4e-10, a, 1.0]
    er, ei = _one(orc, W.KIND_HN, p, om)
    er2, ei2 = _one(orc, W.KIND_CC, [2.7, 5.9, 9.4e-10, a, 0.123], om)  # beta ignored for CC
    ref = np.array([_cole_cole_textbook(w, 2.7, 5.9, 9.4e-10, a) for w in om])
    np.testing.assert_allclose(er, ref[:, 0], rtol=1e-13)
    np.testing.assert_allclose(ei, ref[:, 1], rtol=1e-12, atol=1e-14 * 5.9)
    np.testing.assert_array_equal(er, er2)
    np.testing.assert_array_equal(ei, ei2)


@pytest.mark.parametrize("b", [0.3, 0.45, 0.8, 1.0])
def test_hn_reduces_to_cole_davidson(orc, b):
    om = W.log_grid(1e5, 1e11, 257)
    er, ei = _one(orc, W.KIND_HN, [3.1, 40.0, 2e-9, 1.0, b], om)
    er2, ei2 = _one(orc, W.KIND_CD, [3.1, 40.0, 2e-9, 0.77, b], om)  # alpha ignored for CD
    ref = np.array([_cole_davidson_textbook(w, 3.1, 40.0, 2e-9, b) for w in om])
    np.testing.assert_allclose(er, ref[:, 0], rtol=1e-13)
    np.testing.assert_allclose(ei, ref[:, 1], rtol=1e-12, atol=1e-14 * 40)
    np.testing.assert_array_equal(er, er2)
    np.testing.assert_array_equal(ei, ei2)


def test_hn_reduces_to_debye(orc):
    om = W.log_grid(1e5, 1e11, 101)
    tau = 3.3e-10
    er, ei = _one(orc, W.KIND_HN, [4.0, 11.0, tau, 1.0, 1.0], om)
    x = om * tau
    np.testing.assert_allclose(er, 4.0 + 11.0 / (1 + x * x), rtol=1e-14)
    np.testing.assert_allclose(ei, 11.0 * x / (1 + x * x), rtol=1e-14)


def test_hn_is_lossy_and_limits(orc):
    # eps'' > 0 everywhere (Eq. 1 sign), eps' -> eps_inf + d_eps at low f and -> eps_inf at high f
    om = W.log_grid(1e-2, 1e20, 400)
    er, ei = _one(orc, W.KIND_HN, [2.7, 5.9, 9.4e-10, 0.91, 0.45], om)
    assert np.all(ei > 0)
    assert er[0] == pytest.approx(8.6, rel=1e-4)
    assert er[-1] == pytest.approx(2.7, rel=1e-4)


def test_jonscher_properties(orc):
    om = W.log_grid(1e6, 1e10, 200)
    wp = 2 * math.pi * 1e8
    # n = 1: lossless constant eps_inf + chi
    er, ei = _one(orc, W.KIND_JONSCHER, [3.0, 7.0, wp, 1.0], om)
    np.testing.assert_allclose(er, 10.0, rtol=1e-15)
    np.testing.assert_allclose(ei, 0.0, atol=1e-14)
    for n in (0.1, 0.4, 0.9):
        er, ei = _one(orc, W.KIND_JONSCHER, [3.0, 7.0, wp, n], om)
        assert np.all(ei > 0)
        # constant-Q: loss tangent of the dispersive part is frequency independent
        np.testing.assert_allclose(ei / (er - 3.0), math.tan(math.pi * (1 - n) / 2), rtol=1e-12)
        # power law: log-log slope of eps'' is n - 1; at w = w_p the magnitude is chi
        slope = np.diff(np.log(ei)) / np.diff(np.log(om))
        np.testing.assert_allclose(slope, n - 1, atol=1e-10)
        er1, ei1 = _one(orc, W.KIND_JONSCHER, [3.0, 7.0, wp, n], np.array([wp]))
        assert math.hypot(er1[0] - 3.0, ei1[0]) == pytest.approx(7.0, rel=1e-14)


def test_crim_limits(orc):
    om = W.log_grid(1e6, 1e10, 64)
    water = list(W.WATER)
    er0, ei0 = _one(orc, W.KIND_CRIM, water + [0.0, 6.5], om)
    np.testing.assert_allclose(er0, 6.5, rtol=1e-15)
    np.testing.assert_allclose(ei0, 0.0, atol=1e-15)
    er1, ei1 = _one(orc, W.KIND_CRIM, water + [1.0, 6.5], om)
    erw, eiw = _one(orc, W.KIND_DEBYE, water, om)
    np.testing.assert_allclose(er1, erw, rtol=1e-13)
    np.testing.assert_allclose(ei1, eiw, rtol=1e-12)
    # lossless water limit (tau -> 0): CRIM of two real permittivities is
    # (f sqrt(e1) + (1-f) sqrt(e2))^2
    er, ei = _one(orc, W.KIND_CRIM, [80.0, 0.0, 1e-12, 0.3, 4.0], om)
    np.testing.assert_allclose(er, (0.3 * math.sqrt(80) + 0.7 * 2.0) ** 2, rtol=1e-14)
    # mixture lies between the phases
    er, ei = _one(orc, W.KIND_CRIM, water + [0.25, 6.5], om)
    assert np.all((er > 6.5) & (er < erw)) and np.all(ei > 0) and np.all(ei < eiw)


def test_hnsum_without_noise_is_sum_of_terms(orc):
    om = W.log_grid(1e5, 1e11, 128)
    p = np.zeros(16)
    p[0], p[1] = 3.0, 2
    p[2:6] = [10.0, 1e-9, 0.7, 0.5]
    p[6:10] = [4.0, 1e-11, 0.9, 1.0]
    er, ei = orc.material_eval([W.KIND_HNSUM], p[None], [0, 128], om)
    a_r, a_i = _one(orc, W.KIND_HN, [3.0, 10.0, 1e-9, 0.7, 0.5], om)
    b_r, b_i = _one(orc, W.KIND_HN, [0.0, 4.0, 1e-11, 0.9, 1.0], om)
    np.testing.assert_allclose(er, a_r + b_r, rtol=1e-14)
    np.testing.assert_allclose(ei, a_i + b_i, rtol=1e-14)


def test_hnsum_noise_statistics(orc):
    F = 20000
    om = W.log_grid(1e5, 1e11, F)
    p = np.zeros(16)
    p[0], p[1] = 3.0, 1
    p[2:6] = [10.0, 1e-9, 0.7, 0.5]
    clean_r, clean_i = orc.material_eval([W.KIND_HNSUM], p[None], [0, F], om)
    p[14] = 0.01
    nr, ni = orc.material_eval([W.KIND_HNSUM], p[None], [0, F], om, noise_seed=5)
    e1 = nr / clean_r - 1
    e2 = ni / clean_i - 1
    for e in (e1, e2):
        assert abs(e.mean()) < 4 * 0.01 / math.sqrt(F)
        assert e.std() == pytest.approx(0.01, rel=0.03)
    assert abs(np.corrcoef(e1, e2)[0, 1]) < 0.05
    # deterministic in the seed, different across seeds
    nr2, _ = orc.material_eval([W.KIND_HNSUM], p[None], [0, F], om, noise_seed=5)
    nr3, _ = orc.material_eval([W.KIND_HNSUM], p[None], [0, F], om, noise_seed=6)
    np.testing.assert_array_equal(nr, nr2)
    assert np.any(nr != nr3)


@pytest.mark.parametrize("kind,p", [(W.KIND_HN, [2.7, 5.9, 9.4e-10, 0.91, 0.45]),
                                    (W.KIND_HN, [5.0, 60.0, 1e-8, 0.35, 0.8]),
                                    (W.KIND_CC, [3.0, 20.0, 1e-10, 0.6, 1.0]),
                                    (W.KIND_CD, [3.0, 20.0, 1e-10, 1.0, 0.4]),
                                    (W.KIND_DEBYE, [3.0, 20.0, 1e-10])])
def test_material_jacobian_matches_central_differences(orc, kind, p):
    om = W.log_grid(1e5, 1e11, 41)
    er, ei, J = _one(orc, kind, p, om, jac=True)
    full = [p[0], p[1], p[2], p[3] if len(p) > 3 else 1.0, p[4] if len(p) > 4 else 1.0]
    for q in range(5):
        if kind == W.KIND_DEBYE and q >= 3:
            continue
        if (kind == W.KIND_CC and q == 4) or (kind == W.KIND_CD and q == 3):
            continue  # fixed exponent: not a free parameter of this kind
        h = 1e-6 * abs(full[q])
        pp, pm = list(full), list(full)
        pp[q] += h
        pm[q] -= h
        rp, ip = _one(orc, W.KIND_HN, pp, om)
        rm, im_ = _one(orc, W.KIND_HN, pm, om)
        fd_r = (rp - rm) / (2 * h)
        fd_i = (ip - im_) / (2 * h)
        scale = np.max(np.abs(np.concatenate([fd_r, fd_i]))) + 1e-300
        np.testing.assert_allclose(J[:, q, 0], fd_r, rtol=0, atol=2e-7 * scale)
        np.testing.assert_allclose(J[:, q, 1], fd_i, rtol=0, atol=2e-7 * scale)


def test_unknown_kind_rejected(orc):
    with pytest.raises(ValueError):
        orc.material_eval([9], np.zeros((1, 16)), [0, 3], np.ones(3))


def test_material_sample_equals_full_batch_slices(orc):
    wl = W.tables(M=40, F=64, iters=0)
    er, ei = orc.material_eval(wl.kind, wl.params, wl.f_off, wl.omega, noise_seed=wl.noise_seed)
    idx = np.array([3, 17, 39])
    fo = np.arange(4) * 64
    om = np.concatenate([wl.omega[wl.f_off[m]:wl.f_off[m + 1]] for m in idx])
    e1, e2 = orc.material_eval_sample(wl.kind[idx], wl.params[idx], fo, om, idx, noise_seed=wl.noise_seed)
    np.testing.assert_array_equal(e1, np.concatenate([er[wl.f_off[m]:wl.f_off[m + 1]] for m in idx]))
    np.testing.assert_array_equal(e2, np.concatenate([ei[wl.f_off[m]:wl.f_off[m + 1]] for m in idx]))
