"""Pins of the oracle's differential evolution (DE/rand/1/bin, Storn & Price
1997; the paper's DE-DLS alternative, Sec. III-A): the donors decoded from
trials of a population built to reveal them (distinct, never the target,
uniform), binomial crossover (one coordinate at CR = 0, the expected share
otherwise), the box, greedy selection, and that it finds a brute-force
global minimum."""
import numpy as np

import workloads as W


def _pop(orc, P, N, M=1):
    return orc.Population(P * M, M, N, 8)


def _decode_donors(orc, P, t, seed=3):
    """Row p of the population holds (p, p^2) so that a trial with F = 1 and
    CR = 1 reads u = (r1 + r2 - r3, r1^2 + r2^2 - r3^2), and with F = 0 reads r1."""
    pop = _pop(orc, P, 2)
    p = np.arange(P, dtype=np.float64)
    pop.x[:, 0] = p
    pop.x[:, 1] = p * p
    lb, ub = [-1e9], [1e9]
    orc.de_trial([0, P], [2], lb, ub, 0.0, 0.0, 1.0, seed, t, pop)
    r1 = pop.u[:, 0].copy()
    orc.de_trial([0, P], [2], lb, ub, 1.0, 1.0, 1.0, seed, t, pop)
    dif = pop.u[:, 0] - r1                   # r2 - r3
    dsq = pop.u[:, 1] - r1 * r1              # r2^2 - r3^2
    s = dsq / dif                            # r2 + r3
    r2 = (s + dif) / 2
    r3 = (s - dif) / 2
    return np.stack([r1, r2, r3], 1).astype(np.int64)


def test_donors_distinct_exclude_target_and_uniform(orc):
    P = 7
    counts = np.zeros((P, P))
    for t in range(1, 400):
        r = _decode_donors(orc, P, t)
        for i in range(P):
            assert len(set(r[i])) == 3 and i not in r[i], (t, i, r[i])
            assert np.all((r[i] >= 0) & (r[i] < P))
            counts[i, r[i, 0]] += 1
    # r1 uniform over the P - 1 other members (chi-square, 6 dof per target, 0.1 % level)
    for i in range(P):
        obs = np.delete(counts[i], i)
        exp = obs.sum() / (P - 1)
        chi2 = np.sum((obs - exp) ** 2 / exp)
        assert chi2 < 22.5, (i, chi2)


def test_crossover_one_coordinate_at_cr_zero_and_share_otherwise(orc):
    P, N = 16, 10
    pop = _pop(orc, P, N)
    rng = np.random.default_rng(1)
    pop.x[:] = rng.uniform(-10, -5, size=(P, N))
    pos = np.zeros(N)
    for t in range(1, 200):
        orc.de_trial([0, P], [N], [-1e3], [1e3], 0.5, 1.0, 0.0, 11, t, pop)
        diff = pop.u != pop.x
        assert np.all(diff.sum(1) == 1)
        pos += diff.sum(0)
    # the forced coordinate is uniform over N (chi-square, 9 dof, 0.1 % level)
    exp = pos.sum() / N
    assert np.sum((pos - exp) ** 2 / exp) < 27.9
    share = []
    for t in range(1, 200):
        orc.de_trial([0, P], [N], [-1e3], [1e3], 0.5, 1.0, 0.7, 11, t, pop)
        share.append(np.mean(pop.u != pop.x))
    # expected share CR + (1 - CR)/N = 0.73 (binomial crossover with one forced coordinate)
    assert abs(np.mean(share) - 0.73) < 0.01


def test_mutant_arithmetic_and_degenerate_population(orc):
    # identical members: every difference vector is zero, trial == target
    P, N = 6, 4
    pop = _pop(orc, P, N)
    pop.x[:] = -8.25
    orc.de_trial([0, P], [N], [-12.0], [-6.0], 0.5, 1.0, 1.0, 5, 1, pop)
    assert np.all(pop.u == -8.25)
    # F = 1/2 on a population of exact binary fractions: u = r1 + (r2 - r3)/2 exactly
    pop.x[:] = np.arange(P)[:, None] * 0.25
    r = _decode_donors(orc, P, 9, seed=5)
    orc.de_trial([0, P], [N], [-1e9], [1e9], 0.5, 0.5, 1.0, 5, 9, pop)
    np.testing.assert_array_equal(pop.u[:, 0], 0.25 * r[:, 0] + 0.5 * (0.25 * r[:, 1] - 0.25 * r[:, 2]))


def test_trials_stay_in_the_box(orc):
    P, N = 32, 6
    pop = _pop(orc, P, N)
    orc.de_init([0, P], [N], [-9.0], [-8.0], 2, pop)
    assert np.all((pop.x[:, :N] >= -9.0) & (pop.x[:, :N] <= -8.0))
    redrawn = 0
    for t in range(1, 50):
        orc.de_trial([0, P], [N], [-9.0], [-8.0], 0.9, 1.0, 0.9, 2, t, pop)
        assert np.all((pop.u[:, :N] >= -9.0) & (pop.u[:, :N] <= -8.0))
        redrawn += np.sum(pop.u[:, :N] != pop.x[:, :N])
        pop.x[:] = pop.u
    assert redrawn > 0


def test_selection_is_greedy_and_nan_never_wins(orc):
    P, N = 5, 2
    pop = _pop(orc, P, N)
    orc.de_init([0, P], [N], [-10.0], [-6.0], 4, pop)
    c0 = np.array([3.0, 1.0, np.nan, 2.0, 1.0])
    orc.de_select([0, P], [N], 0, pop.x.copy(), c0, pop)
    assert np.array_equal(pop.fit[[0, 1, 3, 4]], c0[[0, 1, 3, 4]]) and np.isinf(pop.fit[2])
    assert pop.best_idx[0] == 1 and pop.best_cost[0] == 1.0          # lowest index of a tie
    u = pop.x + 0.5
    cu = np.array([3.0, 1.5, 7.0, np.nan, 0.5])                      # equal cost replaces
    x_before = pop.x.copy()
    orc.de_select([0, P], [N], 1, u, cu, pop)
    np.testing.assert_array_equal(pop.x[0], u[0])
    np.testing.assert_array_equal(pop.x[1], x_before[1])
    np.testing.assert_array_equal(pop.x[2], u[2])
    np.testing.assert_array_equal(pop.x[3], x_before[3])
    assert pop.best_idx[0] == 4 and pop.best_cost[0] == 0.5
    np.testing.assert_array_equal(pop.best_x[0, :N], u[4, :N])
    assert pop.history[0, 0] == 1.0 and pop.history[0, 1] == 0.5


def test_small_population_is_not_evolved(orc):
    pop = _pop(orc, 3, 2)
    orc.de_init([0, 3], [2], [-10.0], [-6.0], 1, pop)
    pop.u[:] = 0.0
    orc.de_trial([0, 3], [2], [-10.0], [-6.0], 0.5, 1.0, 0.7, 1, 1, pop)
    np.testing.assert_array_equal(pop.u, pop.x)


def test_de_finds_single_pole_global_minimum(orc):
    om = W.log_grid(1e6, 1e10, 200)
    params = np.zeros((1, 16))
    params[0, :5] = [3.0, 20.0, 1e-9, 0.8, 0.7]
    er, ei = orc.material_eval([W.KIND_HN], params, [0, 200], om)
    grid = np.arange(-12, -7, 1e-4)
    gb = orc.Batch([0, 200], [0, len(grid)], [1], om, er, ei)
    cmin = orc.fit_eval(gb, grid[:, None])[0].min()
    b = orc.Batch([0, 200], [0, 15], [1], om, er, ei)
    pop = orc.de_run(b, [-12.0], [-7.0], 40, seed=0)
    assert pop.best_cost[0] <= cmin * (1 + 1e-6)
    assert np.all(np.diff(pop.history[0]) <= 0)


def test_de_on_the_single_hn_example(orc):
    wl = W.single_hn()
    er, ei = orc.material_eval(wl.kind, wl.params, wl.f_off, wl.omega)
    b = orc.Batch(wl.f_off, [0, 75], wl.n_poles, wl.omega, er, ei)      # 15 x N members
    pop = orc.de_run(b, wl.lb, wl.ub, 150, seed=0)
    ob = orc.Batch(wl.f_off, [0, 1], wl.n_poles, wl.omega, er, ei)
    c, w, e, st = orc.fit_eval(ob, pop.best_x)
    afe = orc.afe(wl.omega, er, ei, w[0], 10.0 ** pop.best_x[0], e[0])
    assert afe < 10.0, afe
