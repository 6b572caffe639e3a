"""Range argument of the cost kernel's grouped basis, checked on the host.

Four poles share one reciprocal in the frequency passes: with d_i = 1 + w^2
tau_i^2 scaled by s = 2^-k (k from the poles' tau at the largest admissible
frequency, w < 1e45, capped at 253, and raised to the largest k of the wave),
the kernel forms p01 = d0 d1, p23 = d2 d3, r = 1/(p01 p23), R0/s = d1 (r p23),
... and U0/s = d1 (w (r p23)).  The claims: for |log10 tau| <= 30, 0 < w <
1e45 and any wave exponent between the lane's own and the cap, every
intermediate is finite and normal, and the results are 1/d and w/d divided by
s to within a few ulp.  Plain float64 products here (the kernel fuses the
first add; the range does not depend on it).
"""
import numpy as np

OMEGA_BOUND = 1e45
TINY = np.finfo(np.float64).tiny


def own_exponent(tau2):
    """k of one group: ceil((sum of frexp exponents of d(1e45)) - 990) / 4, capped at 253."""
    e = np.frexp(1.0 + OMEGA_BOUND * OMEGA_BOUND * tau2)[1].sum(axis=-1)
    k = np.where(e > 990, (e - 990 + 3) >> 2, 0)
    return np.minimum(k, 253)


def grouped(w, tau2, k):
    """The kernel's operation order for one group; returns (R/s, U/s, intermediates)."""
    s = np.ldexp(1.0, -k)[..., None]
    d = w[..., None] ** 2 * (tau2 * s) + s
    p01, p23 = d[..., 0] * d[..., 1], d[..., 2] * d[..., 3]
    p = p01 * p23
    r = 1.0 / p
    r01, r23 = r * p23, r * p01
    R = np.stack([d[..., 1] * r01, d[..., 0] * r01, d[..., 3] * r23, d[..., 2] * r23], axis=-1)
    u01, u23 = w * r01, w * r23
    U = np.stack([d[..., 1] * u01, d[..., 0] * u01, d[..., 3] * u23, d[..., 2] * u23], axis=-1)
    return R, U, [d, p01, p23, p, r, r01, r23, u01, u23, R, U]


def _draw(n, rng):
    theta = rng.uniform(-30.0, 30.0, size=(n, 4))
    # edge cases: every pole at either end, one pole at each end
    theta[: n // 8] = 30.0
    theta[n // 8: n // 4] = -30.0
    theta[n // 4: 3 * n // 8, :2] = 30.0
    tau2 = (10.0 ** theta) ** 2
    w = 10.0 ** rng.uniform(-30.0, np.log10(OMEGA_BOUND) - 1e-9, size=n)
    return tau2, w


def test_scales_stay_in_bounds():
    rng = np.random.default_rng(1)
    tau2, _ = _draw(200_000, rng)
    k = own_exponent(tau2)
    assert k.min() >= 0 and k.max() <= 252          # valid inputs never reach the cap
    # s^4 prod d(1e45) <= 2^990 with the lane's own k
    lp = np.log2(1.0 + OMEGA_BOUND ** 2 * tau2).sum(axis=-1) - 4 * k
    assert lp.max() <= 990.0 + 1e-9


def test_intermediates_finite_and_normal_for_any_wave_exponent():
    rng = np.random.default_rng(2)
    tau2, w = _draw(200_000, rng)
    k_own = own_exponent(tau2)
    for k_wave in (k_own, np.full_like(k_own, 253), rng.integers(k_own, 254)):
        with np.errstate(over="raise", under="ignore", invalid="raise", divide="raise"):
            R, U, inter = grouped(w, tau2, k_wave)
        for v in inter:   # every intermediate is positive, finite and normal
            assert np.all(np.isfinite(v))
            assert np.all(v >= TINY)
        s = np.ldexp(1.0, -k_wave)[..., None]
        d = 1.0 + w[..., None] ** 2 * tau2
        # R/s and U/s against the direct forms, a few ulp
        relR = np.abs(R * s * d - 1.0)
        relU = np.abs(U * s * d / w[..., None] - 1.0)
        assert relR.max() < 16 * np.finfo(np.float64).eps
        assert relU.max() < 16 * np.finfo(np.float64).eps


def test_rejected_lane_does_not_push_the_wave_out_of_range():
    # a rejected candidate (|log10 tau| > 30) alone would ask for k > 253; the cap
    # keeps the wave's exponent at 253, which the valid lanes tolerate
    tau2_bad = np.full((1, 4), (10.0 ** 100) ** 2)
    assert own_exponent(tau2_bad)[0] == 253
    rng = np.random.default_rng(3)
    tau2, w = _draw(50_000, rng)
    with np.errstate(over="raise", under="ignore", invalid="raise", divide="raise"):
        R, U, inter = grouped(w, tau2, np.full(len(w), 253))
    assert all(np.all(np.isfinite(v)) and np.all(v >= TINY) for v in inter)


def test_odd_pole_shared_by_two_points():
    """The pole left over after the groups and pairs (outside the scaled
    groups, d = 1 + w^2 tau^2 unscaled) takes one reciprocal for two points a
    and b: r = 1/(d_a d_b), R_a = d_b r, R_b = d_a r, U_a = w_a (d_b r).
    Over the whole admissible range the product stays finite (d < 1e150) and
    the values are within a few ulp of 1/d and w/d."""
    rng = np.random.default_rng(4)
    n = 200_000
    tau2 = (10.0 ** rng.uniform(-30.0, 30.0, size=n)) ** 2
    tau2[: n // 8] = 1e60          # the largest admissible tau
    tau2[n // 8: n // 4] = 1e-60   # the smallest
    w = 10.0 ** rng.uniform(-30.0, np.log10(OMEGA_BOUND) - 1e-9, size=(n, 2))
    w[: n // 16] = OMEGA_BOUND * (1 - 1e-12)
    with np.errstate(over="raise", under="ignore", invalid="raise", divide="raise"):
        d = w ** 2 * tau2[:, None] + 1.0
        p = d[:, 0] * d[:, 1]
        r = 1.0 / p
        R = np.stack([d[:, 1] * r, d[:, 0] * r], axis=1)
        U = w * R
    for v in (d, p, r, R, U):
        assert np.all(np.isfinite(v)) and np.all(v >= TINY)
    eps = np.finfo(np.float64).eps
    assert np.abs(R * d - 1.0).max() < 8 * eps
    assert np.abs(U * d / w - 1.0).max() < 8 * eps
