"""A swarm fit replayed from a captured HIP graph equals the eager fit bit for
bit, on every replay, with eager work and synchronisations between replays;
the eager fit equals the step-by-step calls; and a GPU swarm fit of the single
HN workload reaches the oracle's swarm result."""
import numpy as np
import pytest

import workloads as W
from _helpers import small_ragged, targets_oracle

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


def _snapshot(sw, cost):
    import torch
    torch.cuda.synchronize()
    return {k: getattr(sw, k).cpu().numpy().copy() for k in ("x", "v", "pbest_x", "pbest_cost", "gbest_x",
                                                              "gbest_cost", "gbest_idx", "history")} | {
        "cost": cost.cpu().numpy().copy()}


def _equal(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


@pytest.mark.parametrize("which", ["mixed", "ragged"])
def test_graph_replay_equals_eager(D, orc, which):
    import torch
    if which == "mixed":
        wl = W.mixed_uniform(M=24, F=300, N=8, P=64, iters=12, seed=4)
    else:
        wl = small_ragged(30, seed=13, Fr=(40, 400), Nr=(2, 20), Pr=(16, 130))
        wl.iters = 9
    er, ei = targets_oracle(orc, wl)
    b = D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, _t(er), _t(ei))
    plan = D.Plan(b)
    lb, ub = _t(wl.lb), _t(wl.ub)
    iters = wl.iters
    # step-by-step reference
    sw0 = D.Swarm.empty(wl.P, wl.M, wl.ld, iters + 1)
    D.pso_init(b, lb, ub, sw0, seed=5)
    cost = D.fit_eval(plan, b, sw0.x, want_weights=False)[0]
    for t in range(1, iters + 1):
        D.pso_step(b, lb, ub, sw0, t, True, cost, seed=5)
        cost = D.fit_eval(plan, b, sw0.x, want_weights=False)[0]
    D.pso_step(b, lb, ub, sw0, iters + 1, False, cost, seed=5)
    ref = _snapshot(sw0, cost)
    # eager whole-fit entry point
    sw1 = D.Swarm.empty(wl.P, wl.M, wl.ld, iters + 1)
    c1 = D.pso_run(plan, b, lb, ub, sw1, iters, seed=5, use_graph=False)
    _equal(ref, _snapshot(sw1, c1))
    # graph replays, three times, with unrelated eager work in between
    sw2 = D.Swarm.empty(wl.P, wl.M, wl.ld, iters + 1)
    for rep in range(3):
        c2 = D.pso_run(plan, b, lb, ub, sw2, iters, seed=5, use_graph=True)
        _equal(ref, _snapshot(sw2, c2))
        junk = D.fit_eval(plan, b, _t(W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, rep)))[0]
        torch.cuda.synchronize()
        assert torch.isfinite(junk).any()


def test_graph_recaptured_after_schedule_change(D, orc):
    """A plan re-tiled (new split, autotune) after a captured swarm fit must
    not replay the old graph: the replay equals an eager fit on the new
    schedule."""
    import torch
    wl = small_ragged(20, seed=21, Fr=(40, 300), Nr=(3, 12), Pr=(16, 100))
    er, ei = targets_oracle(orc, wl)
    b = D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, _t(er), _t(ei))
    plan = D.Plan(b)
    lb, ub = _t(wl.lb), _t(wl.ub)
    iters = 6
    sw = D.Swarm.empty(wl.P, wl.M, wl.ld, iters + 1)
    D.pso_run(plan, b, lb, ub, sw, iters, seed=3, use_graph=True)
    theta = _t(W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, 8))
    for change in ("split", "autotune", "split back"):
        if change == "split":
            plan.set_freq_split(4)
        elif change == "autotune":
            plan.set_freq_split(0)   # back to automatic, then measured
            plan.autotune(b, theta, reps=1)
        else:
            plan.set_freq_split(1)
        sw_e = D.Swarm.empty(wl.P, wl.M, wl.ld, iters + 1)
        ce = D.pso_run(plan, b, lb, ub, sw_e, iters, seed=3, use_graph=False)
        ref = _snapshot(sw_e, ce)
        c = D.pso_run(plan, b, lb, ub, sw, iters, seed=3, use_graph=True)
        _equal(ref, _snapshot(sw, c))
        torch.cuda.synchronize()


def test_gpu_swarm_fit_matches_oracle_swarm(D, orc):
    wl = W.single_hn()
    er, ei = targets_oracle(orc, wl)
    ob = orc.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, er, ei)
    osw = orc.pso_run(ob, wl.lb, wl.ub, wl.iters, seed=0)
    b = D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, _t(er), _t(ei))
    sw = D.Swarm.empty(wl.P, wl.M, wl.ld, wl.iters + 1)
    D.pso_run(D.Plan(b), b, _t(wl.lb), _t(wl.ub), sw, wl.iters, seed=0, use_graph=True)
    gh = sw.history.cpu().numpy()[0]
    oh = osw.history[0]
    # identical decisions unless two particles' costs tie within the cost
    # tolerance; report where (if at all) the trajectories part
    same = np.isclose(gh, oh, rtol=1e-9, atol=0)
    first = int(np.argmin(same)) if not same.all() else None
    print(f"single HN swarm: GPU {gh[-1]:.10e} oracle {oh[-1]:.10e}; histories identical up to "
          f"{first if first is not None else 'the end'}")
    assert same[: min(10, len(same))].all()
    assert gh[-1] <= oh[0] and abs(gh[-1] - oh[-1]) <= 0.05 * oh[-1]
