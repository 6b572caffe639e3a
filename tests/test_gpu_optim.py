"""GPU parity of the swarm, the adjoint, the autograd wrappers and the polish
against the oracle, plus a full-size sampled check of the cost kernel in the
benchmark's launch configuration."""
import numpy as np
import pytest

import workloads as W
from _helpers import (COST_RTOL, attributed_cost_err, cost_floor, cost_rel_err, mixed_scale_workload, small_ragged,
                      small_uniform, targets_oracle)

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


def _batch(D, wl, er, ei):
    return D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, _t(er), _t(ei))


@pytest.mark.parametrize("which", ["single", "ragged"])
def test_pso_bit_exact_lockstep(D, orc, which):
    """The swarm update is bit-reproducible: fed the same costs, GPU and oracle
    produce identical positions, velocities and bests at every iteration."""
    import torch
    if which == "single":
        wl = W.single_hn()
        iters = 50
    else:
        wl = small_ragged(12, seed=21, Fr=(30, 200), Nr=(1, 24), Pr=(1, 90))
        iters = 15
    er, ei = targets_oracle(orc, wl)
    ob = orc.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, er, ei)
    b = _batch(D, wl, er, ei)
    ld = wl.ld
    osw = orc.Swarm(wl.P, wl.M, ld, iters + 1)
    gsw = D.Swarm.empty(wl.P, wl.M, ld, iters + 1)
    lb, ub = _t(wl.lb), _t(wl.ub)
    orc.pso_init(wl.cand_off, wl.n_poles, wl.lb, wl.ub, 7, osw)
    D.pso_init(b, lb, ub, gsw, wl.inertia, wl.c1, wl.c2, 7)

    def same(t):
        torch.cuda.synchronize()
        for name in ("x", "v", "pbest_x", "pbest_cost", "gbest_cost", "gbest_idx"):
            g = getattr(gsw, name).cpu().numpy()
            o = getattr(osw, name)
            if name in ("x", "v", "pbest_x"):
                for m in range(wl.M):
                    a, e, n = wl.cand_off[m], wl.cand_off[m + 1], wl.n_poles[m]
                    assert np.array_equal(g[a:e, :n], o[a:e, :n]), f"{name} differs at t={t}, material {m}"
            else:
                assert np.array_equal(g, o), f"{name} differs at t={t}"
        for m in range(wl.M):
            if osw.gbest_idx[m] >= 0:
                assert np.array_equal(gsw.gbest_x.cpu().numpy()[m, :wl.n_poles[m]], osw.gbest_x[m, :wl.n_poles[m]])

    same(0)
    for t in range(1, iters + 2):
        cost = orc.fit_eval(ob, osw.x)[0]
        move = t <= iters
        orc.pso_step(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.inertia, wl.c1, wl.c2, 7, t, move, cost, osw)
        D.pso_step(b, lb, ub, gsw, t, move, _t(cost), wl.inertia, wl.c1, wl.c2, 7)
        same(t)
    np.testing.assert_array_equal(gsw.history.cpu().numpy(), osw.history)


def test_gpu_swarm_is_deterministic_and_finds_good_fits(D, orc):
    import torch
    wl = W.single_hn()
    er, ei = targets_oracle(orc, wl)
    b = _batch(D, wl, er, ei)
    plan = D.Plan(b)
    runs = []
    for _ in range(2):
        sw = D.Swarm.empty(wl.P, wl.M, wl.ld, wl.iters + 1)
        lb, ub = _t(wl.lb), _t(wl.ub)
        D.pso_init(b, lb, ub, sw, seed=0)
        cost = D.fit_eval(plan, b, sw.x, want_weights=False)[0]
        for t in range(1, wl.iters + 1):
            D.pso_step(b, lb, ub, sw, t, True, cost, seed=0)
            cost = D.fit_eval(plan, b, sw.x, want_weights=False)[0]
        D.pso_step(b, lb, ub, sw, wl.iters + 1, False, cost, seed=0)
        torch.cuda.synchronize()
        runs.append((sw.gbest_x.cpu().numpy().copy(), sw.history.cpu().numpy().copy()))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    h = runs[0][1][0]
    assert np.all(np.diff(h) <= 0) and h[-1] < h[0]
    # the fitted model is a useful approximation (average fractional error, Sec. IV)
    ob = orc.Batch(wl.f_off, [0, 1], wl.n_poles, wl.omega, er, ei)
    c, w, e, st = orc.fit_eval(ob, runs[0][0])
    afe = orc.afe(wl.omega, er, ei, w[0], 10.0 ** runs[0][0][0], e[0])
    print(f"single HN: gbest cost {h[-1]:.4e}, average fractional error {afe:.2f} %")
    assert afe < 10.0


@pytest.mark.parametrize("N,F,flags,damping", [(5, 120, 0, 1e-8), (8, 300, 0, 1e-8), (8, 300, 1, 1e-8),
                                               (10, 300, 0, 1e-8), (11, 350, 0, 1e-8), (12, 400, 0, 1e-8),
                                               (14, 400, 0, 1e-8), (16, 500, 0, 1e-8), (20, 600, 0, 1e-8),
                                               (6, 200, 0, 1e-4)])
def test_adjoint_matches_oracle(D, orc, N, F, flags, damping):
    import torch
    wl = small_uniform(3, F, N, 20, seed=N * 7 + F)
    er, ei = targets_oracle(orc, wl)
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=3)
    gc = np.linspace(0.5, 2.0, wl.P)
    ob = orc.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, er, ei)
    oc, og, ogr, ogi, ost = orc.fit_grad(ob, theta, damping=damping, flags=flags, grad_cost=gc)
    b = _batch(D, wl, er, ei)
    plan = D.Plan(b, target_grads=True)
    c, g, gr, gi, st = D.fit_eval_grad(plan, b, _t(theta), damping=damping, flags=flags, grad_cost=_t(gc),
                                      targets=True)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    np.testing.assert_array_equal(st.cpu().numpy(), ost)
    rel = cost_rel_err(c.cpu().numpy(), oc, cost_floor(wl, er, ei))
    rel, _ = attributed_cost_err(orc, ob, theta, c.cpu().numpy(), cost_floor(wl, er, ei), damping, flags, rel)
    assert rel.max() <= COST_RTOL
    # gradient: relative to each candidate's largest component
    gerr = np.max(np.abs(g - og), axis=1) / np.max(np.abs(og), axis=1)
    print(f"N={N} F={F}: max theta-gradient rel err {gerr.max():.2e}")
    assert np.all(gerr <= 1e-6)
    for a, o in ((gr.cpu().numpy(), ogr), (gi.cpu().numpy(), ogi)):
        for m in range(wl.M):
            s, e = wl.f_off[m], wl.f_off[m + 1]
            assert np.max(np.abs(a[s:e] - o[s:e])) <= 1e-6 * np.max(np.abs(o[s:e]))



@pytest.mark.parametrize("N", [4, 8, 12, 20])
def test_adjoint_mixed_scale_waves(D, orc, N):
    """The adjoint where the ordinary band and a band 33 decades down share
    waves (the frequency passes then run the ordinary lanes at group scales
    near 2^-200): costs, theta-gradients and target gradients against the
    oracle."""
    import torch
    wl = mixed_scale_workload(N)
    er, ei = targets_oracle(orc, wl)
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=5)
    gc = np.linspace(0.5, 2.0, wl.P)
    ob = orc.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, er, ei)
    oc, og, ogr, ogi, ost = orc.fit_grad(ob, theta, grad_cost=gc)
    b = _batch(D, wl, er, ei)
    plan = D.Plan(b, target_grads=True)
    c, g, gr, gi, st = D.fit_eval_grad(plan, b, _t(theta), grad_cost=_t(gc), targets=True)
    torch.cuda.synchronize()
    print(f"[adjoint mixed-scale N{N}] plan={plan.info()}", flush=True)
    np.testing.assert_array_equal(st.cpu().numpy(), ost)
    rel = cost_rel_err(c.cpu().numpy(), oc, cost_floor(wl, er, ei))
    rel, _ = attributed_cost_err(orc, ob, theta, c.cpu().numpy(), cost_floor(wl, er, ei), 1e-8, 0, rel)
    assert rel.max() <= COST_RTOL
    g = g.cpu().numpy()
    gerr = np.max(np.abs(g - og), axis=1) / np.max(np.abs(og), axis=1)
    print(f"[adjoint mixed-scale N{N}] max theta-gradient rel err {gerr.max():.2e}", flush=True)
    assert np.all(gerr <= 1e-6)
    for a, o in ((gr.cpu().numpy(), ogr), (gi.cpu().numpy(), ogi)):
        for m in range(wl.M):
            s, e = wl.f_off[m], wl.f_off[m + 1]
            assert np.max(np.abs(a[s:e] - o[s:e])) <= 1e-6 * np.max(np.abs(o[s:e]))

def test_adjoint_ragged_matches_oracle(D, orc):
    """Several pole counts at once (their buckets run on concurrent streams),
    with the target gradients summed per material."""
    import torch
    wl = small_ragged(18, seed=31, Fr=(40, 300), Nr=(1, 24), Pr=(0, 40))
    er, ei = targets_oracle(orc, wl)
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=8)
    gc = np.linspace(0.5, 2.0, wl.P)
    ob = orc.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, er, ei)
    oc, og, ogr, ogi, ost = orc.fit_grad(ob, theta, grad_cost=gc)
    b = _batch(D, wl, er, ei)
    plan = D.Plan(b, target_grads=True)
    c, g, gr, gi, st = D.fit_eval_grad(plan, b, _t(theta), grad_cost=_t(gc), targets=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(st.cpu().numpy(), ost)
    rel = cost_rel_err(c.cpu().numpy(), oc, cost_floor(wl, er, ei))
    rel, _ = attributed_cost_err(orc, ob, theta, c.cpu().numpy(), cost_floor(wl, er, ei), 1e-8, 0, rel)
    assert rel.max() <= COST_RTOL
    g = g.cpu().numpy()
    for cI in range(wl.P):
        m = int(np.searchsorted(wl.cand_off, cI, side="right") - 1)
        n = wl.n_poles[m]
        assert np.max(np.abs(g[cI, :n] - og[cI, :n])) <= 1e-6 * np.max(np.abs(og[cI, :n])), cI
    for a, o in ((gr.cpu().numpy(), ogr), (gi.cpu().numpy(), ogi)):
        for m in range(wl.M):
            s, e = wl.f_off[m], wl.f_off[m + 1]
            if wl.cand_off[m + 1] == wl.cand_off[m]:
                assert np.all(a[s:e] == 0.0)
            else:
                assert np.max(np.abs(a[s:e] - o[s:e])) <= 1e-6 * np.max(np.abs(o[s:e])), m


def test_adjoint_matches_central_differences_on_gpu(D, orc):
    import torch
    wl = small_uniform(1, 2000, 12, 1, seed=4, fmin=1e5, fmax=1e11, kinds=[W.KIND_HN])
    er, ei = targets_oracle(orc, wl)
    th = np.array([[-12.5, -11.7, -11.0, -10.3, -9.6, -9.0, -8.4, -7.9, -7.4, -6.9, -6.5, -6.2]])
    st, z, _, _, _ = orc.fit_detail(wl.omega, er, ei, th[0])
    assert np.min(np.abs(z)) > 1e-3 * np.max(np.abs(z))
    b = _batch(D, wl, er, ei)
    _, g, _, _, _ = D.fit_eval_grad(D.Plan(b), b, _t(th))
    h = 1e-6
    pts = np.repeat(th, 24, axis=0)
    for i in range(12):
        pts[2 * i, i] += h
        pts[2 * i + 1, i] -= h
    bb = D.Batch(wl.f_off, [0, 24], wl.n_poles, wl.omega, _t(er), _t(ei))
    c = D.fit_eval(D.Plan(bb), bb, _t(pts), want_weights=False)[0].cpu().numpy()
    fd = (c[0::2] - c[1::2]) / (2 * h)
    g = g.cpu().numpy()[0]
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())


def test_autograd_functions(D, orc):
    import torch
    wl = small_uniform(4, 300, 6, 8, seed=9, kinds=[W.KIND_HN, W.KIND_CC])
    er, ei, J = orc.material_eval(wl.kind, wl.params, wl.f_off, wl.omega, jac=True)
    b = _batch(D, wl, er, ei)
    plan = D.Plan(b, target_grads=True)
    theta = _t(W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=1)).requires_grad_(True)
    params = _t(wl.params).requires_grad_(True)
    kind = torch.tensor(wl.kind, device="cuda")
    er_t, ei_t = D.HNTarget.apply(params, kind, b)
    cost = D.DebyeCost.apply(theta, er_t, ei_t, plan, b)
    wts = torch.linspace(1, 2, wl.P, dtype=torch.float64, device="cuda")
    (cost * wts).sum().backward()
    # reference: oracle adjoint + Jacobian chain rule
    ob = orc.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, er, ei)
    _, og, ogr, ogi, _ = orc.fit_grad(ob, theta.detach().cpu().numpy(), grad_cost=wts.cpu().numpy())
    np.testing.assert_allclose(theta.grad.cpu().numpy(), og, rtol=1e-6, atol=1e-7 * np.abs(og).max())
    gp = params.grad.cpu().numpy()
    for m in range(wl.M):
        s, e = wl.f_off[m], wl.f_off[m + 1]
        ref = J[s:e, :, 0].T @ ogr[s:e] + J[s:e, :, 1].T @ ogi[s:e]
        np.testing.assert_allclose(gp[m, :5], ref, rtol=1e-6, atol=1e-9 * np.abs(ref).max())
        assert np.all(gp[m, 5:] == 0)
        # exact invariant: the fitted eps_inf absorbs the material's eps_inf
        assert abs(gp[m, 0]) <= 1e-8 * np.abs(ref).max()


def test_polish_matches_oracle_behaviour(D, orc):
    import torch
    wl = W.hn_cc(M=6, F=400, N=8, P=48, iters=12, seed=5)
    er, ei = targets_oracle(orc, wl)
    b = _batch(D, wl, er, ei)
    plan = D.Plan(b)
    sw = D.Swarm.empty(wl.P, wl.M, wl.ld, wl.iters + 1)
    lb, ub = _t(wl.lb), _t(wl.ub)
    D.pso_init(b, lb, ub, sw, seed=2)
    cost = D.fit_eval(plan, b, sw.x, want_weights=False)[0]
    for t in range(1, wl.iters + 1):
        D.pso_step(b, lb, ub, sw, t, True, cost, seed=2)
        cost = D.fit_eval(plan, b, sw.x, want_weights=False)[0]
    D.pso_step(b, lb, ub, sw, wl.iters + 1, False, cost, seed=2)
    th0 = sw.gbest_x.cpu().numpy().copy()
    # include a swarm best on the box corner (duplicate poles at the bound)
    th0[0, :] = wl.lb[0]
    th0[0, 1] = wl.ub[0]
    b1 = D.Batch(wl.f_off, np.arange(wl.M + 1), wl.n_poles, wl.omega, b.eps_re, b.eps_im)
    th = _t(th0)
    hist = D.lbfgs_polish(b1, th, lb, ub, steps=25).cpu().numpy()
    ob1 = orc.Batch(wl.f_off, np.arange(wl.M + 1), wl.n_poles, wl.omega, er, ei)
    oth, ohist = orc.lbfgs(ob1, th0, wl.lb, wl.ub, steps=25)
    gth = th.cpu().numpy()
    print("GPU polish", hist[:, 0], "->", hist[:, -1])
    print("oracle polish", ohist[:, 0], "->", ohist[:, -1])
    assert np.all(np.diff(hist, axis=1) <= 0)
    assert np.all(gth >= wl.lb[0]) and np.all(gth <= wl.ub[0])
    np.testing.assert_allclose(hist[:, 0], ohist[:, 0], rtol=1e-10)
    # the first step takes the same decision on both sides; afterwards the
    # paths may part where the Gram matrix is near-singular (material 0 starts
    # on the box corner), so well-conditioned materials are compared closely
    # and every material must make progress
    np.testing.assert_allclose(hist[:, 1], ohist[:, 1], rtol=1e-6)
    np.testing.assert_allclose(hist[1:, -1], ohist[1:, -1], rtol=1e-5)
    assert np.all(hist[:, -1] < hist[:, 0])
    # the cost reported at the end is the cost of the returned point
    c = orc.fit_eval(ob1, gth)[0]
    np.testing.assert_allclose(c, hist[:, -1], rtol=1e-9)


def test_full_size_sampled_parity_bench_configuration(D, orc):
    """All 262144 candidates of the mixed workload in one launch (the bench's
    plan); 4096 sampled candidates checked one by one against the oracle."""
    import torch
    wl = W.mixed_uniform(M=1024, F=1000, N=8, P=256, iters=1, seed=0)
    er, ei = targets_oracle(orc, wl)
    b = _batch(D, wl, er, ei)
    plan = D.Plan(b)
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=91)
    c, w, e, st = D.fit_eval(plan, b, _t(theta))
    torch.cuda.synchronize()
    c = c.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(wl.P, 4096, replace=False))
    mats = idx // 256
    sub = orc.Batch(np.arange(len(idx) + 1) * 1000, np.arange(len(idx) + 1), np.full(len(idx), 8),
                    np.concatenate([wl.omega[wl.f_off[m]:wl.f_off[m + 1]] for m in mats]),
                    np.concatenate([er[wl.f_off[m]:wl.f_off[m + 1]] for m in mats]),
                    np.concatenate([ei[wl.f_off[m]:wl.f_off[m + 1]] for m in mats]))
    oc = orc.fit_eval(sub, theta[idx])[0]
    floor = cost_floor(wl, er, ei)[idx]
    stats = {}
    rel, _ = attributed_cost_err(orc, sub, theta[idx], c[idx], floor, 1e-8, 0, cost_rel_err(c[idx], oc, floor),
                                 stats)
    print(f"full-size sample: {stats}")
    assert rel.max() <= COST_RTOL
