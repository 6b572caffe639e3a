"""Pins of the oracle's annealing (generalized simulated annealing, Tsallis &
Stariolo 1996; the paper's DA-DLS alternative, Sec. III-A): its own exp and
log against the library ones, the visiting variate against the Student-t
distribution, the temperature schedule's closed form, the acceptance rule,
the periodic box, and that it finds a brute-force global minimum."""
import numpy as np
import pytest
from scipy import stats

import workloads as W


def test_series_exp_log_accuracy(orc):
    x = np.concatenate([np.linspace(-700, 700, 20001), np.linspace(-1, 1, 2001), [0.0, 1e-300, -1e-300]])
    ex, _ = orc.series_exp_log(x)
    ref = np.exp(x)
    assert np.max(np.abs(ex - ref) / ref) < 4e-16
    y = np.concatenate([np.geomspace(1e-300, 1e300, 20001), np.linspace(0.5, 2, 2001)])
    _, lg = orc.series_exp_log(y)
    ref = np.log(y)
    exact1 = y == 1.0
    assert np.all(lg[exact1] == 0.0)
    err = np.abs(lg - ref)[~exact1] / np.abs(ref[~exact1])
    assert np.max(err) < 6e-16
    ex, lg = orc.series_exp_log([0.0, np.inf, -np.inf, np.nan, -1.0])
    assert lg[0] == -np.inf and lg[1] == np.inf and np.isnan(lg[3]) and np.isnan(lg[4])
    assert ex[0] == 1.0 and ex[1] == np.inf and ex[2] == 0.0


@pytest.mark.parametrize("nu", [0.2346, 1.0, 5.0])
def test_visiting_variate_is_student_t(orc, nu):
    g = orc.student_t(3, 40000, nu)
    ks = stats.kstest(g, stats.t(df=nu).cdf)
    assert ks.pvalue > 1e-3, ks
    assert np.all(np.isfinite(g))


def test_temperature_schedule(orc):
    qv, t0 = 2.62, 5230.0
    for t in (1, 2, 10, 100, 1000):
        vs, ta = orc.da_temps(t, qv, t0)
        T = t0 * (2 ** (qv - 1) - 1) / ((1 + t) ** (qv - 1) - 1)
        assert ta == pytest.approx(T / t, rel=1e-14)
        assert vs == pytest.approx(T ** (1 / (3 - qv)) / np.sqrt(3 - qv), rel=1e-14)
    assert orc.da_temps(1, qv, t0)[1] == pytest.approx(t0, rel=1e-15)     # T(1) = T0


def _one_chain_pop(orc, N=2, P=1, hist=4):
    return orc.Population(P, 1, N, hist)


def test_acceptance_rule(orc):
    qv, qa, t0 = 2.62, -5.0, 5230.0
    P = 4000
    pop = orc.Population(P, 1, 1, 4)
    orc.da_init([0, P], [1], [-10.0], [-6.0], 1, pop)
    orc.da_accept([0, P], [1], 1, 0, pop.x.copy(), np.full(P, 10.0), pop, qv, qa, t0)
    assert np.all(pop.fit == 10.0) and pop.best_idx[0] == 0
    _, ta = orc.da_temps(2, qv, t0)
    # a fixed uphill step dE: accepted with probability (1 - (1 - qa) dE / Ta)^(1/(1-qa))
    dE = 0.05 * ta
    y = pop.x + 0.5
    orc.da_accept([0, P], [1], 1, 2, y, np.full(P, 10.0 + dE), pop, qv, qa, t0)
    p = (1 - (1 - qa) * dE / ta) ** (1 / (1 - qa))
    frac = np.mean(pop.fit == 10.0 + dE)
    assert abs(frac - p) < 4 * np.sqrt(p * (1 - p) / P), (frac, p)
    # downhill always, uphill beyond the cut-off never, NaN never
    pop2 = orc.Population(3, 1, 1, 4)
    orc.da_init([0, 3], [1], [-10.0], [-6.0], 2, pop2)
    orc.da_accept([0, 3], [1], 2, 0, pop2.x.copy(), np.array([5.0, 5.0, 5.0]), pop2, qv, qa, t0)
    cut = ta / (1 - qa)
    orc.da_accept([0, 3], [1], 2, 2, pop2.x + 1, np.array([4.0, 5.0 + 1.01 * cut, np.nan]), pop2, qv, qa, t0)
    np.testing.assert_array_equal(pop2.fit, [4.0, 5.0, 5.0])
    assert pop2.best_idx[0] == 0 and pop2.best_cost[0] == 4.0 and pop2.history[0, 2] == 4.0


def test_proposals_wrap_into_the_box(orc):
    P, N = 200, 5
    pop = orc.Population(P, 1, N, 4)
    orc.da_init([0, P], [N], [-9.0], [-8.0], 5, pop)
    for t in (1, 2, 50):
        orc.da_visit([0, P], [N], [-9.0], [-8.0], 5, t, pop)
        assert np.all((pop.u >= -9.0) & (pop.u <= -8.0))
    # early, hot generations move far: some proposals wrapped around
    orc.da_visit([0, P], [N], [-9.0], [-8.0], 5, 1, pop)
    assert np.mean(np.abs(pop.u - pop.x)) > 0.1


def test_da_finds_single_pole_global_minimum(orc):
    om = W.log_grid(1e6, 1e10, 200)
    params = np.zeros((1, 16))
    params[0, :5] = [3.0, 20.0, 1e-9, 0.8, 0.7]
    er, ei = orc.material_eval([W.KIND_HN], params, [0, 200], om)
    grid = np.arange(-12, -7, 1e-4)
    gb = orc.Batch([0, 200], [0, len(grid)], [1], om, er, ei)
    cmin = orc.fit_eval(gb, grid[:, None])[0].min()
    b = orc.Batch([0, 200], [0, 16], [1], om, er, ei)
    pop = orc.da_run(b, [-12.0], [-7.0], 60, seed=0)
    # annealing locates the basin; the gradient polish then reaches the minimum
    th, hist = orc.lbfgs(orc.Batch([0, 200], [0, 1], [1], om, er, ei), pop.best_x, -12.0, -7.0, steps=20)
    assert hist[0, -1] <= cmin * (1 + 1e-6)
    assert np.all(np.diff(pop.history[0]) <= 0)
