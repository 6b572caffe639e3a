"""Pins of the oracle's counter-based RNG (against numpy's Philox), the particle
swarm (a hand-worked step and invariants) and the L-BFGS polish."""
import math

import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("ctr,key", [([0, 0, 0, 0], [0, 0]), ([5, 7, 11, 2], [123, 456]),
                                     ([2**64 - 1, 3, 2**63, 1], [2**64 - 2, 99])])
def test_philox_matches_numpy(orc, ctr, key):
    # numpy's Philox is 4x64-10; it advances the counter before producing a block
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(ctr, dtype=np.uint64))
    want = bg.random_raw(4)
    c1 = list(ctr)
    c1[0] = (c1[0] + 1) % 2**64
    if c1[0] == 0:
        c1[1] = (c1[1] + 1) % 2**64
    got = orc.philox4x64_10(c1, key)
    np.testing.assert_array_equal(got, want)


def _u01(r):
    return float(int(r) >> 11) * 2.0 ** -53


def test_pso_hand_worked_two_particles(orc):
    # one material, two particles, one dimension
    cand_off = [0, 2]
    n_poles = [1]
    lb, ub = [-12.0], [-6.0]
    seed = 42
    sw = orc.Swarm(2, 1, 1, 4)
    orc.pso_init(cand_off, n_poles, lb, ub, seed, sw)
    for p in range(2):
        r = orc.philox4x64_10([0, p, 0, 0], [seed, 0])
        assert sw.x[p, 0] == -12.0 + 6.0 * _u01(r[0])
        assert sw.v[p, 0] == 6.0 * (2.0 * _u01(r[1]) - 1.0)
        assert sw.pbest_x[p, 0] == sw.x[p, 0]
    assert np.all(sw.pbest_cost == np.inf) and sw.gbest_cost[0] == np.inf and sw.gbest_idx[0] == -1
    x0, v0 = sw.x.copy(), sw.v.copy()
    cost = np.array([3.0, 2.0])
    orc.pso_step(cand_off, n_poles, lb, ub, 0.7, 1.5, 1.5, seed, 1, True, cost, sw)
    assert list(sw.pbest_cost) == [3.0, 2.0]
    assert sw.gbest_cost[0] == 2.0 and sw.gbest_idx[0] == 1 and sw.gbest_x[0, 0] == x0[1, 0]
    assert sw.history[0, 0] == 2.0
    for p in range(2):
        r = orc.philox4x64_10([0, p, 1, 1], [seed, 0])
        r1, r2 = _u01(r[0]), _u01(r[1])
        vel = 0.7 * v0[p, 0]
        vel = vel + (1.5 * r1) * (x0[p, 0] - x0[p, 0])
        vel = vel + (1.5 * r2) * (x0[1, 0] - x0[p, 0])
        assert sw.v[p, 0] == vel
        assert sw.x[p, 0] == min(max(x0[p, 0] + vel, -12.0), -6.0)
    # ties: equal costs keep the earlier best; lower index wins among equals
    x1 = sw.x.copy()
    orc.pso_step(cand_off, n_poles, lb, ub, 0.7, 1.5, 1.5, seed, 2, False, np.array([2.0, 2.0]), sw)
    assert list(sw.pbest_cost) == [2.0, 2.0]
    assert sw.pbest_x[0, 0] == x1[0, 0] and sw.pbest_x[1, 0] == x0[1, 0]
    assert sw.gbest_idx[0] == 1          # not strictly better: gbest unchanged
    assert np.array_equal(sw.x, x1)      # bests-only step does not move
    sw2 = orc.Swarm(2, 1, 1, 4)
    orc.pso_init(cand_off, n_poles, lb, ub, seed, sw2)
    orc.pso_step(cand_off, n_poles, lb, ub, 0.7, 1.5, 1.5, seed, 1, False, np.array([5.0, 5.0]), sw2)
    assert sw2.gbest_idx[0] == 0
    # NaN never becomes a best
    sw3 = orc.Swarm(2, 1, 1, 4)
    orc.pso_init(cand_off, n_poles, lb, ub, seed, sw3)
    orc.pso_step(cand_off, n_poles, lb, ub, 0.7, 1.5, 1.5, seed, 1, True, np.array([np.nan, np.nan]), sw3)
    assert np.all(sw3.pbest_cost == np.inf) and sw3.gbest_idx[0] == -1
    assert np.all(np.isfinite(sw3.x))


def test_pso_invariants_and_resume(orc):
    wl = W.mixed_uniform(M=3, F=120, N=4, P=24, iters=12, seed=1)
    er, ei = orc.material_eval(wl.kind, wl.params, wl.f_off, wl.omega)
    b = orc.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, er, ei)
    sw = orc.pso_run(b, wl.lb, wl.ub, wl.iters, seed=3)
    assert np.all(sw.x >= wl.lb[0]) and np.all(sw.x <= wl.ub[0])
    h = sw.history
    assert np.all(np.diff(h, axis=1) <= 0)                      # gbest never worsens
    for m in range(wl.M):
        a, e = wl.cand_off[m], wl.cand_off[m + 1]
        assert sw.gbest_cost[m] == sw.pbest_cost[a:e].min()
        c = orc.fit_eval(orc.Batch(wl.f_off[m:m + 2] - wl.f_off[m], [0, 1], wl.n_poles[m:m + 1],
                                   wl.omega[wl.f_off[m]:wl.f_off[m + 1]], er[wl.f_off[m]:wl.f_off[m + 1]],
                                   ei[wl.f_off[m]:wl.f_off[m + 1]]), sw.gbest_x[m:m + 1])[0]
        assert c[0] == sw.gbest_cost[m]
    # counter-based RNG: stopping and resuming from saved state is bit-exact
    s1 = orc.Swarm(b.P, b.M, 4, 13)
    orc.pso_init(b.cand_off, b.n_poles, wl.lb, wl.ub, 3, s1)
    cost = orc.fit_eval(b, s1.x)[0]
    for t in range(1, 7):
        orc.pso_step(b.cand_off, b.n_poles, wl.lb, wl.ub, 0.7, 1.5, 1.5, 3, t, True, cost, s1)
        cost = orc.fit_eval(b, s1.x)[0]
    saved, saved_cost = s1.copy(), cost.copy()
    for t in range(7, 13):
        orc.pso_step(b.cand_off, b.n_poles, wl.lb, wl.ub, 0.7, 1.5, 1.5, 3, t, True, saved_cost, saved)
        saved_cost = orc.fit_eval(b, saved.x)[0]
    orc.pso_step(b.cand_off, b.n_poles, wl.lb, wl.ub, 0.7, 1.5, 1.5, 3, 13, False, saved_cost, saved)
    np.testing.assert_array_equal(saved.x, sw.x)
    np.testing.assert_array_equal(saved.gbest_cost, sw.gbest_cost)


def test_pso_finds_single_pole_global_minimum(orc):
    om = W.log_grid(1e6, 1e10, 200)
    params = np.zeros((1, 16))
    params[0, :5] = [3.0, 20.0, 1e-9, 0.8, 0.7]
    er, ei = orc.material_eval([W.KIND_HN], params, [0, 200], om)
    grid = np.arange(-12, -7, 1e-4)
    gb = orc.Batch([0, 200], [0, len(grid)], [1], om, er, ei)
    cmin = orc.fit_eval(gb, grid[:, None])[0].min()
    b = orc.Batch([0, 200], [0, 20], [1], om, er, ei)
    sw = orc.pso_run(b, [-12.0], [-7.0], 30, seed=0)
    assert sw.gbest_cost[0] <= cmin * (1 + 1e-6)
    # polishing from there keeps it at the grid minimum with a vanishing gradient
    th, hist = orc.lbfgs(orc.Batch([0, 200], [0, 1], [1], om, er, ei), sw.gbest_x, -12.0, -7.0, steps=10)
    assert hist[0, -1] <= cmin
    _, g, _, _, _ = orc.fit_grad(orc.Batch([0, 200], [0, 1], [1], om, er, ei), th)
    assert abs(g[0, 0]) < 1e-6 * hist[0, -1]


def test_lbfgs_monotone_and_improves(orc):
    wl = W.hn_cc(M=3, F=300, N=6, P=32, iters=10, seed=2)
    er, ei = orc.material_eval(wl.kind, wl.params, wl.f_off, wl.omega)
    b = orc.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, er, ei)
    sw = orc.pso_run(b, wl.lb, wl.ub, wl.iters, seed=5)
    bm = orc.Batch(wl.f_off, np.arange(wl.M + 1), wl.n_poles, wl.omega, er, ei)
    th, hist = orc.lbfgs(bm, sw.gbest_x, wl.lb, wl.ub, steps=30)
    assert np.all(np.diff(hist, axis=1) <= 0)
    assert np.all(th >= wl.lb[0]) and np.all(th <= wl.ub[0])
    assert np.all(hist[:, -1] < 0.9 * hist[:, 0])
    c = orc.fit_eval(bm, th)[0]
    np.testing.assert_array_equal(c, hist[:, -1])


def test_lbfgs_stays_in_box_from_a_corner(orc):
    # a swarm best on the corner of the box (many poles at the bound): the
    # polish must stay inside the box and never increase the cost
    om = W.log_grid(1e6, 1e10, 400)
    params = np.zeros((1, 16))
    params[0, :5] = [3.0, 40.0, 3e-9, 0.5, 0.6]
    er, ei = orc.material_eval([W.KIND_HN], params, [0, 400], om)
    th0 = np.array([[-12.0, -7.0, -12.0, -12.0, -12.0, -12.0, -12.0, -12.0]])
    b = orc.Batch([0, 400], [0, 1], [8], om, er, ei)
    th, hist = orc.lbfgs(b, th0, -12.0, -7.0, steps=40)
    assert np.all(th >= -12.0) and np.all(th <= -7.0)
    assert np.all(np.diff(hist[0]) <= 0) and hist[0, -1] < hist[0, 0]


def _dense_bfgs_inverse(S, Y):
    """Inverse-Hessian approximation by explicit BFGS updates from gamma I
    (gamma = s.y / y.y of the newest pair), pairs applied oldest first:
    H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T (Nocedal & Wright,
    eq. 6.17 / 7.19, with the initial scaling of eq. 7.20)."""
    n, N = S.shape
    gamma = S[-1] @ Y[-1] / (Y[-1] @ Y[-1]) if n else 1.0
    H = gamma * np.eye(N)
    for s, y in zip(S, Y):
        rho = 1.0 / (s @ y)
        V = np.eye(N) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return H


@pytest.mark.parametrize("N,n", [(1, 1), (4, 2), (6, 5), (12, 10), (20, 3)])
def test_lbfgs_two_loop_equals_dense_bfgs(orc, N, n):
    """The polish's search direction: the two-loop product H v equals the
    dense BFGS inverse built from the same pairs, H is symmetric positive
    definite, and it satisfies the newest secant condition H y = s."""
    g = np.random.default_rng(N * 31 + n)
    A = g.standard_normal((N, N))
    A = A @ A.T + N * np.eye(N)                 # SPD curvature: s.y > 0
    S = g.standard_normal((n, N))
    Y = S @ A.T + 0.1 * g.standard_normal((n, N))
    assert np.all(np.einsum("ij,ij->i", S, Y) > 0)
    H = _dense_bfgs_inverse(S, Y)
    v = g.standard_normal(N)
    hv = orc.lbfgs_two_loop(S, Y, v)
    np.testing.assert_allclose(hv, H @ v, rtol=1e-11, atol=1e-12 * np.abs(H @ v).max())
    # the two-loop operator itself, column by column
    Hop = np.stack([orc.lbfgs_two_loop(S, Y, e) for e in np.eye(N)], axis=1)
    np.testing.assert_allclose(Hop, Hop.T, rtol=0, atol=1e-11 * np.abs(Hop).max())
    assert np.linalg.eigvalsh(0.5 * (Hop + Hop.T)).min() > 0
    np.testing.assert_allclose(orc.lbfgs_two_loop(S, Y, Y[-1]), S[-1], rtol=1e-11, atol=1e-12 * np.abs(S[-1]).max())


def test_lbfgs_two_loop_without_pairs_is_identity(orc):
    v = np.array([0.3, -2.0, 5.5])
    np.testing.assert_array_equal(orc.lbfgs_two_loop(np.zeros((0, 3)), np.zeros((0, 3)), v), v)


def test_lbfgs_two_loop_pins_order_and_scaling(orc):
    """Plausible slips in the recursion (pairs taken newest-first in the dense
    update, the scaling from the oldest pair, no scaling) give a different
    product, so the comparison above would catch them."""
    g = np.random.default_rng(7)
    N, n = 5, 4
    A = g.standard_normal((N, N))
    A = A @ A.T + N * np.eye(N)
    S = g.standard_normal((n, N))
    Y = S @ A.T + 0.3 * g.standard_normal((n, N))
    v = g.standard_normal(N)
    hv = orc.lbfgs_two_loop(S, Y, v)
    wrong_order = _dense_bfgs_inverse(S[::-1], Y[::-1]) @ v
    gamma_old = (S[0] @ Y[0]) / (Y[0] @ Y[0])
    H = gamma_old * np.eye(N)
    for s, y in zip(S, Y):
        rho = 1.0 / (s @ y)
        V = np.eye(N) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    for other in (wrong_order, H @ v):
        assert np.max(np.abs(hv - other)) > 1e-6 * np.max(np.abs(hv))
