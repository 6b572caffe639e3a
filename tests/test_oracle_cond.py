"""Pins of the oracle's FP64-sensitivity measure (the condition number of the
cost under componentwise relative perturbations of the basis), used to judge
ill-conditioned candidates: its derivatives against central differences of
the cost computed from an explicitly perturbed basis, its invariances, and
the first-order bound it states."""
import numpy as np
import pytest

import workloads as W


def _hn(orc, p, om):
    params = np.zeros((1, 16))
    params[0, :5] = p
    return orc.material_eval([W.KIND_HN], params, [0, len(om)], om)


def _basis(orc, om, th):
    re, im = orc.basis(om, th)
    return re.T.copy(), im.T.copy()      # [F][N]


CASES = [
    ([3.0, 20.0, 1e-9, 0.7, 0.6], [-11.1, -9.7, -8.6, -7.4], 1e-8, 0),
    ([5.5, 60.0, 3e-10, 0.4, 0.9], [-11.5, -10.6, -9.9, -9.0, -8.1, -7.2], 1e-8, 0),
    ([4.0, 30.0, 5e-9, 0.8, 0.3], [-11.0, -9.1, -8.8, -7.5, -10.2], 1e-4, 1),
    # a near-duplicate pair of relaxation times (the ill-conditioned case)
    ([3.4, 15.0, 1e-9, 0.8, 0.6], [-10.9, -7.0, -9.3, -9.3004, -8.2], 1e-8, 0),
]


@pytest.mark.parametrize("p,th,lam,flags", CASES)
def test_basis_derivatives_match_central_differences(orc, p, th, lam, flags):
    om = W.log_grid(1e6, 1e10, 60)
    er, ei = _hn(orc, p, om)
    th = np.array(th)
    cond, dR, dI, st = orc.fit_cond(om, er, ei, th, lam, flags)
    assert st == 0 and np.isfinite(cond) and cond > 0
    R, I = _basis(orc, om, th)
    c0, _ = orc.fit_from_basis(R, I, er, ei, lam, flags, precision=80)
    scale = max(np.max(np.abs(dR * R)), np.max(np.abs(dI * I)))
    rng = np.random.default_rng(3)
    F, N = R.shape
    for _ in range(12):
        k, i = int(rng.integers(F)), int(rng.integers(N))
        for B, dB in ((R, dR), (I, dI)):
            h = 1e-6 * abs(B[k, i])
            Bp, Bm = B.copy(), B.copy()
            Bp[k, i] += h
            Bm[k, i] -= h
            args = (Bp, I) if B is R else (R, Bp)
            cp = orc.fit_from_basis(*args, er, ei, lam, flags, precision=80)[0]
            args = (Bm, I) if B is R else (R, Bm)
            cm = orc.fit_from_basis(*args, er, ei, lam, flags, precision=80)[0]
            fd = (cp - cm) / (2 * h)
            # compared on the scale of the contributions |dC/dB * B|
            assert abs(fd - dB[k, i]) * abs(B[k, i]) <= 1e-5 * scale + 1e-7 * abs(fd * B[k, i]), (k, i)
    # the sum that defines cond
    assert cond == pytest.approx((np.abs(dR * R).sum() + np.abs(dI * I).sum()) / c0, rel=1e-10)


def test_cond_is_scale_invariant_and_bounds_perturbations(orc):
    om = W.log_grid(1e6, 1e10, 80)
    er, ei = _hn(orc, [3.4, 15.0, 1e-9, 0.8, 0.6], om)
    th = np.array([-10.9, -7.0, -9.3, -9.3004, -8.2])
    cond, _, _, _ = orc.fit_cond(om, er, ei, th)
    cond2, _, _, _ = orc.fit_cond(om, 7.0 * er, 7.0 * ei, th)
    assert cond2 == pytest.approx(cond, rel=1e-9)
    # componentwise relative perturbations of size eta move the cost by at most
    # eta * cond * C to first order (eta small enough to stay first order)
    R, I = _basis(orc, om, th)
    c0 = orc.fit_from_basis(R, I, er, ei, precision=80)[0]
    rng = np.random.default_rng(9)
    eta = 1e-12
    worst = 0.0
    for _ in range(20):
        Rp = R * (1 + eta * rng.choice([-1.0, 1.0], size=R.shape))
        Ip = I * (1 + eta * rng.choice([-1.0, 1.0], size=I.shape))
        c = orc.fit_from_basis(Rp, Ip, er, ei, precision=80)[0]
        worst = max(worst, abs(c - c0) / c0)
    assert worst <= 1.05 * eta * cond
    assert worst >= 1e-4 * eta * cond       # not vacuous: random signs reach a fair share of it


def test_fit_from_basis_reproduces_fit_eval(orc):
    om = W.log_grid(1e5, 1e10, 50)
    er, ei = _hn(orc, [3.4, 15.0, 1e-9, 0.8, 0.6], om)
    th = np.array([-11.5, -10.0, -8.7, -7.9, -6.5])
    R, I = _basis(orc, om, th)
    b = orc.Batch([0, len(om)], [0, 1], [5], om, er, ei)
    for prec in (64, 80):
        c_ref = orc.fit_eval(b, th[None], precision=prec)[0][0]
        c, st = orc.fit_from_basis(R, I, er, ei, precision=prec)
        assert st == 0
        if prec == 64:
            assert c == c_ref          # same arithmetic on the same basis
        else:
            assert c == pytest.approx(c_ref, rel=1e-14)


def test_judge_costs_tiers(orc):
    """The judgement accepts exactly: errors within rtol of the FP64 oracle or
    within rtol of the 80-bit oracle.  An error beyond both fails and is
    reported as the error against the 80-bit result, even where it is within
    the cost's FP64 rounding sensitivity (planted on the CPU)."""
    # a CRIM mixture with two relaxation times 5e-4 decades apart
    om = W.log_grid(1e6, 1e10, 267)
    params = np.zeros((1, 16))
    params[0, :5] = [4.9, 75.0, 9.2e-12, 0.154, 6.95]
    er, ei = orc.material_eval([W.KIND_CRIM], params, [0, len(om)], om)
    th = np.array([[-10.938, -7.034, -11.2767, -8.984, -11.2772]])
    b = orc.Batch([0, len(om)], [0, 1], [5], om, er, ei)
    c64 = orc.fit_eval(b, th)[0]
    c80 = orc.fit_eval(b, th, precision=80)[0]
    cond = orc.fit_cond(om, er, ei, th[0])[0]
    floor = np.array([0.0])
    bound = cond * orc.UNIT_ROUNDOFF
    assert bound > 1e-10          # this candidate is ill-conditioned in FP64
    # within the FP64 rounding sensitivity but beyond both oracles: fails
    x = c80 * (1 + 0.5 * bound)
    assert abs(x - c64) / c64 > 1e-10
    bad, st = orc.judge_costs(b, th, x, c64, floor, 1e-10)
    assert bad[0] == pytest.approx(0.5 * bound, rel=1e-3) and st["failed"] == 1 and st["oracle_limited"] == 0
    assert st["over"][0][0] == 0 and st["over"][0][3] == pytest.approx(bound)
    # within rtol of the 80-bit oracle only: passes as oracle-limited, error vs 80-bit
    y = c80 * (1 + 5e-11)
    if abs(y - c64) / c64 > 1e-10:
        ok, st = orc.judge_costs(b, th, y, c64, floor, 1e-10)
        assert ok[0] == pytest.approx(5e-11, rel=1e-3) and st["oracle_limited"] == 1 and st["failed"] == 0
    near, st = orc.judge_costs(b, th, c64 * (1 + 1e-11), c64, floor, 1e-10)
    assert near[0] <= 1e-10 and st["oracle_limited"] == 0 and st["failed"] == 0


def _domain_batch(orc, N, seed, lo, hi, M=3, P=40):
    wl_kind, wl_params = W.draw_mixed(M, seed, 1e6, 1e10)
    om = W.log_grid(1e6, 1e10, 120)
    er, ei = orc.material_eval(wl_kind, wl_params, W.offsets([len(om)] * M), np.tile(om, M))
    b = orc.Batch(W.offsets([len(om)] * M), W.offsets([P] * M), np.full(M, N), np.tile(om, M), er, ei)
    th = np.random.default_rng(seed).uniform(lo, hi, (M * P, N))
    return b, th


@pytest.mark.parametrize("N", [3, 8])
def test_oracle_precisions_inside_the_search_box(orc, N):
    """Inside a workload's search box the three instances of the oracle agree
    with binary128 within a modest multiple (the Householder solve adds its
    own rounding on F = 120 rows) of the cost's sensitivity to rounding the
    basis at their precision: cond * 2^-64 for the 80-bit instance (at most a
    few 1e-12 here), cond * 2^-53 for FP64."""
    lb, ub = W.tau_bounds(1e6, 1e10)
    b, th = _domain_batch(orc, N, 5 + N, lb, ub)
    c64, c80, c128 = (orc.fit_eval(b, th, precision=p)[0] for p in (64, 80, 128))
    r80 = np.abs(c80 - c128) / c128
    r64 = np.abs(c64 - c128) / c128
    cond = orc.fit_cond_batch(b, th)
    assert r80.max() <= 1e-11
    assert np.all(r80 <= 1e-14 + 100 * cond * 2.0 ** -64)
    assert np.all(r64 <= 1e-13 + 100 * cond * orc.UNIT_ROUNDOFF)


def test_oracle_precisions_far_out_of_band(orc):
    """Over the whole admissible range (|log10 tau| <= 30, poles up to 20
    decades outside the band) the cost is not determined to 1e-10 by FP64
    arithmetic: the FP64 oracle is off from the binary128 instance by orders
    of magnitude on many candidates, the 80-bit instance far less, and the
    FP64 oracle's error follows the cost's FP64 sensitivity cond * u."""
    b, th = _domain_batch(orc, 8, 3, -30.0, 30.0)
    c64, c80, c128 = (orc.fit_eval(b, th, precision=p)[0] for p in (64, 80, 128))
    st = orc.fit_eval(b, th)[3]
    ok = st == 0
    r64 = (np.abs(c64 - c128) / c128)[ok]
    r80 = (np.abs(c80 - c128) / c128)[ok]
    cond = orc.fit_cond_batch(b, th)[ok]
    assert np.mean(r64 > 1e-10) > 0.5          # FP64 cannot hold the tolerance out there
    assert r64.max() > 1.0                      # ... and is off by more than the cost itself
    assert np.median(r80) < 1e-3 * np.median(r64)
    # where FP64 is off by more than 1e-10, its cost is that sensitive to the basis rounding
    over = r64 > 1e-10
    assert np.all(cond[over] * orc.UNIT_ROUNDOFF > 1e-12)
