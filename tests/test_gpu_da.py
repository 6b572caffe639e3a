"""Annealing on the GPU (generalized simulated annealing, batched Markov
chains): bit-exact lockstep with the oracle when fed the same costs (its
series exp and log included), the whole-fit entry point equal to the
step-by-step calls, its graph replays equal to eager launches, and a GPU fit
of the single HN example against the oracle's."""
import numpy as np
import pytest

import workloads as W
from _helpers import small_ragged, targets_oracle

pytestmark = pytest.mark.gpu

DA = dict(qv=2.62, qa=-5.0, t0=5230.0)


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


def _cases():
    single = W.single_hn()
    single.cand_off = np.array([0, 48])
    ragged = small_ragged(14, seed=23, Fr=(30, 200), Nr=(1, 24), Pr=(5, 70))
    P = np.diff(ragged.cand_off)
    P[[1, 4, 8]] = [1, 0, 3]              # a single chain, empty, a few chains
    ragged.cand_off = W.offsets(P)
    return {"single": (single, 40), "ragged": (ragged, 12)}


@pytest.mark.parametrize("which", ["single", "ragged"])
def test_da_bit_exact_lockstep(D, orc, which):
    import torch
    wl, iters = _cases()[which]
    er, ei = targets_oracle(orc, wl)
    ob = orc.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, er, ei)
    b = D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, _t(er), _t(ei))
    ld = wl.ld
    P, M = int(wl.cand_off[-1]), wl.M
    op = orc.Population(P, M, ld, iters + 1)
    gp = D.Population.empty(P, M, ld, iters + 1)
    lb, ub = _t(wl.lb), _t(wl.ub)
    orc.da_init(wl.cand_off, wl.n_poles, wl.lb, wl.ub, 9, op)
    D.da_init(b, lb, ub, gp, seed=9, **DA)

    def same(t, names=("x", "fit", "best_cost", "best_idx")):
        torch.cuda.synchronize()
        for name in names:
            g = getattr(gp, name).cpu().numpy()
            o = getattr(op, name)
            if g.ndim == 2:
                for m in range(M):
                    a, e, n = wl.cand_off[m], wl.cand_off[m + 1], wl.n_poles[m]
                    assert np.array_equal(g[a:e, :n], o[a:e, :n]), f"{name} differs at t={t}, material {m}"
            else:
                assert np.array_equal(g, o, equal_nan=True), f"{name} differs at t={t}"
        for m in range(M):
            if op.best_idx[m] >= 0:
                assert np.array_equal(gp.best_x.cpu().numpy()[m, :wl.n_poles[m]], op.best_x[m, :wl.n_poles[m]])

    same(-1)
    cost = orc.fit_eval(ob, op.x)[0]
    orc.da_accept(wl.cand_off, wl.n_poles, 9, 0, op.x.copy(), cost, op)
    D.da_accept(b, gp, 0, gp.x.clone(), _t(cost), seed=9, **DA)
    same(0)
    for t in range(1, iters + 1):
        orc.da_visit(wl.cand_off, wl.n_poles, wl.lb, wl.ub, 9, t, op)
        D.da_visit(b, lb, ub, gp, t, seed=9, **DA)
        torch.cuda.synchronize()
        gu = gp.u.cpu().numpy()
        for m in range(M):
            a, e, n = wl.cand_off[m], wl.cand_off[m + 1], wl.n_poles[m]
            assert np.array_equal(gu[a:e, :n], op.u[a:e, :n]), f"proposal differs at t={t}, material {m}"
        cost = orc.fit_eval(ob, op.u)[0]
        orc.da_accept(wl.cand_off, wl.n_poles, 9, t, op.u, cost, op)
        D.da_accept(b, gp, t, gp.u, _t(cost), seed=9, **DA)
        same(t)
    np.testing.assert_array_equal(gp.history.cpu().numpy(), op.history)


@pytest.mark.parametrize("which", ["single", "ragged"])
def test_da_run_equals_steps_and_graph_replays(D, orc, which):
    import torch
    wl, iters = _cases()[which]
    er, ei = targets_oracle(orc, wl)
    b = D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, _t(er), _t(ei))
    plan = D.Plan(b)
    lb, ub = _t(wl.lb), _t(wl.ub)
    P, M, ld = int(wl.cand_off[-1]), wl.M, wl.ld
    # step by step through the primitive calls
    ref = D.Population.empty(P, M, ld, iters + 1)
    D.da_init(b, lb, ub, ref, seed=4, **DA)
    c = D.fit_eval(plan, b, ref.x, want_weights=False)[0]
    D.da_accept(b, ref, 0, ref.x.clone(), c, seed=4, **DA)
    for t in range(1, iters + 1):
        D.da_visit(b, lb, ub, ref, t, seed=4, **DA)
        c = D.fit_eval(plan, b, ref.u, want_weights=False)[0]
        D.da_accept(b, ref, t, ref.u, c, seed=4, **DA)
    torch.cuda.synchronize()
    keys = ("x", "fit", "best_x", "best_cost", "best_idx", "history")
    want = {k: getattr(ref, k).cpu().numpy().copy() for k in keys}
    for use_graph in (False, True, True, True):
        pop = D.Population.empty(P, M, ld, iters + 1)
        D.da_run(plan, b, lb, ub, pop, iters, seed=4, use_graph=use_graph, **DA)
        torch.cuda.synchronize()
        for k in keys:
            assert np.array_equal(getattr(pop, k).cpu().numpy(), want[k], equal_nan=True), (use_graph, k)
        # unrelated eager work between replays
        junk = D.fit_eval(plan, b, _t(W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, ld, 3)))[0]
        torch.cuda.synchronize()
        assert torch.isfinite(junk).any()


def test_gpu_da_fit_matches_oracle_fit(D, orc):
    wl, _ = _cases()["single"]
    iters = 150
    er, ei = targets_oracle(orc, wl)
    ob = orc.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, er, ei)
    opop = orc.da_run(ob, wl.lb, wl.ub, iters, seed=0)
    b = D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, _t(er), _t(ei))
    pop = D.Population.empty(int(wl.cand_off[-1]), 1, wl.ld, iters + 1)
    D.da_run(D.Plan(b), b, _t(wl.lb), _t(wl.ub), pop, iters, seed=0)
    gh = pop.history.cpu().numpy()[0]
    oh = opop.history[0]
    same = np.isclose(gh, oh, rtol=1e-9, atol=0)
    first = int(np.argmin(same)) if not same.all() else None
    print(f"single HN DA: GPU {gh[-1]:.10e} oracle {oh[-1]:.10e}; histories identical up to "
          f"{first if first is not None else 'the end'}")
    assert same[:10].all()
    assert gh[-1] <= oh[0] and abs(gh[-1] - oh[-1]) <= 0.05 * oh[-1]
    # the annealing's best, polished by the gradient local search
    b1 = D.Batch(wl.f_off, [0, 1], wl.n_poles, wl.omega, _t(er), _t(ei))
    th = pop.best_x.clone()
    D.lbfgs_polish(b1, th, _t(wl.lb), _t(wl.ub), steps=50)
    c, w, e, st = orc.fit_eval(orc.Batch(wl.f_off, [0, 1], wl.n_poles, wl.omega, er, ei), th.cpu().numpy())
    afe = orc.afe(wl.omega, er, ei, w[0], 10.0 ** th.cpu().numpy()[0], e[0])
    print(f"single HN DA + polish: average fractional error {afe:.2f} %")
    assert afe < 10.0
