"""DEBYE_FLAG_DD_REFINE: the refinement step in double-double arithmetic.

The flag changes only how accurately the damped least-squares weights of
Sec. III-B are computed, so its results are judged against the oracle without
the flag.  The checks:
  - whole workloads in the launch configuration the bench uses (one plan,
    autotuned schedule), every candidate judged: the mixed N = 8 batch with
    the bench's parity candidates (where the FP64 refinement leaves a few
    candidates in 10^6 between 1e-10 and 3e-10 of the 80-bit oracle) and the
    first 512 materials of the ragged workload (pole counts 2..20, all three
    pole splits): no candidate beyond 1e-10 of the FP64 or 80-bit oracle;
  - a persistent-launch plan evaluates the flag with per-bucket launches:
    results bit-identical to a per-bucket plan's;
  - swarm, differential-evolution and annealing runs with the flag record the
    flag's costs;
  - the flag's exclusions: together with DEBYE_FLAG_NO_REFINE, in the adjoint,
    in the polish and in the autograd function."""
import numpy as np
import pytest

import workloads as W
from _helpers import COST_RTOL, cost_floor, targets_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    import paper_2109_01928_amd as D

    assert torch.cuda.is_available()
    D.lib()
    return D


def _first_materials(wl, K):
    import dataclasses
    f1 = int(wl.f_off[K])
    return dataclasses.replace(wl, name=f"{wl.name} first {K}", kind=wl.kind[:K], params=wl.params[:K],
                               f_off=wl.f_off[:K + 1], omega=wl.omega[:f1], n_poles=wl.n_poles[:K],
                               cand_off=wl.cand_off[:K + 1], lb=wl.lb[:K], ub=wl.ub[:K])


def _batch(D, wl, er, ei):
    import torch
    return D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, torch.tensor(er, device="cuda"),
                   torch.tensor(ei, device="cuda"))


def _judge_all(D, orc, wl, theta_seed, tag):
    import torch
    er, ei = targets_oracle(orc, wl)
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=theta_seed)
    b = _batch(D, wl, er, ei)
    plan = D.Plan(b)
    th = torch.tensor(theta, device="cuda")
    plan.autotune(b, th, reps=1)
    print(f"[{tag}] {wl.P} candidates, schedule {plan.info()}", flush=True)
    c_def, _, _, st_def = D.fit_eval(plan, b, th, want_weights=False)
    c_dd, _, _, st_dd = D.fit_eval(plan, b, th, flags=D.FLAG_DD_REFINE, want_weights=False)
    torch.cuda.synchronize()
    ob = orc.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, er, ei)
    c64, _, _, ost = orc.fit_eval(ob, theta)
    np.testing.assert_array_equal(st_dd.cpu().numpy(), ost)
    np.testing.assert_array_equal(st_def.cpu().numpy(), ost)
    floor = cost_floor(wl, er, ei)
    rel_def, s_def = orc.judge_costs(ob, theta, c_def.cpu().numpy(), c64, floor, COST_RTOL)
    rel_dd, s_dd = orc.judge_costs(ob, theta, c_dd.cpu().numpy(), c64, floor, COST_RTOL)
    for what, r, st in (("FP64", rel_def, s_def), ("double-double", rel_dd, s_dd)):
        print(f"[{tag}] {what} refinement: max {r.max():.3e}; {st['oracle_limited'] + st['failed']} judged vs "
              f"80-bit (max error there {st['max_rel_80']:.3e}), failed {st['failed']} {st['over'][:4]}", flush=True)
    assert s_dd["failed"] == 0 and rel_dd.max() <= COST_RTOL
    return rel_def, rel_dd


def test_dd_refine_whole_mixed_batch(D, orc):
    wl = W.mixed_uniform(M=1024, F=1000, N=8, P=256, iters=1, seed=0)
    _judge_all(D, orc, wl, 77, "mixed")


def test_dd_refine_ragged_materials(D, orc):
    full = W.mixed_ragged(M=4096, iters=1)
    wl = _first_materials(full, 512)
    assert set(np.unique(wl.n_poles)) == set(range(2, 21))
    _judge_all(D, orc, wl, 77, "ragged 512")


def test_dd_refine_persistent_plan_and_swarm(D, orc):
    import torch
    wl = W.mixed_ragged(M=48, iters=1, seed=5, fmax_points=600)
    er, ei = targets_oracle(orc, wl)
    theta = torch.tensor(W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=5), device="cuda")
    b = _batch(D, wl, er, ei)
    pb, pp = D.Plan(b), D.Plan(b)
    pb.set_launch(D.LAUNCH_BUCKETS)
    pp.set_launch(D.LAUNCH_PERSISTENT)
    out_b = D.fit_eval(pb, b, theta, flags=D.FLAG_DD_REFINE)
    out_p = D.fit_eval(pp, b, theta, flags=D.FLAG_DD_REFINE)
    torch.cuda.synchronize()
    # weights: the columns of each candidate's own poles (the rest are not written)
    npc = torch.tensor(np.repeat(wl.n_poles, np.diff(wl.cand_off)), device="cuda")
    used = torch.arange(wl.ld, device="cuda")[None, :] < npc[:, None]
    for i, (x, y) in enumerate(zip(out_b, out_p)):
        if i == 1:
            x, y = x[used], y[used]
        assert torch.equal(torch.nan_to_num(x, nan=-7.0), torch.nan_to_num(y, nan=-7.0)), i
    # a swarm run with the flag: the recorded best costs are the flag's costs
    # of the recorded best positions
    lb = torch.tensor(wl.lb, device="cuda")
    ub = torch.tensor(wl.ub, device="cuda")
    sw = D.Swarm.empty(wl.P, wl.M, wl.ld, 6)
    D.pso_run(pb, b, lb, ub, sw, 5, 0.7, 1.5, 1.5, 3, flags=D.FLAG_DD_REFINE)
    c_best = D.fit_eval(pb, b, sw.pbest_x, flags=D.FLAG_DD_REFINE, want_weights=False)[0]
    torch.cuda.synchronize()
    ok = torch.isfinite(sw.pbest_cost)
    assert ok.any()
    assert torch.equal(c_best[ok], sw.pbest_cost[ok])
    # the same for differential evolution and annealing: the fitness they keep
    # for their current members is the flag's cost of those members
    for run in (D.de_run, D.da_run):
        pop = D.Population.empty(wl.P, wl.M, wl.ld, 6)
        run(pb, b, lb, ub, pop, 5, seed=4, flags=D.FLAG_DD_REFINE)
        c_now = D.fit_eval(pb, b, pop.x, flags=D.FLAG_DD_REFINE, want_weights=False)[0]
        torch.cuda.synchronize()
        ok = torch.isfinite(pop.fit)
        assert ok.any(), run.__name__
        assert torch.equal(c_now[ok], pop.fit[ok]), run.__name__


def test_dd_refine_flag_rules(D, orc):
    import torch
    wl = W.mixed_uniform(M=4, F=120, N=6, P=16, iters=1, seed=3)
    er, ei = targets_oracle(orc, wl)
    b = _batch(D, wl, er, ei)
    plan = D.Plan(b)
    th = torch.tensor(W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=3), device="cuda")
    with pytest.raises(D.DebyeError):
        D.fit_eval(plan, b, th, flags=D.FLAG_DD_REFINE | D.FLAG_NO_REFINE)
    with pytest.raises(D.DebyeError):
        D.fit_eval_grad(plan, b, th, flags=D.FLAG_DD_REFINE)
    b1 = D.Batch(wl.f_off, np.arange(wl.M + 1), wl.n_poles, wl.omega, b.eps_re, b.eps_im)
    pol = D.Polish(b1, wl.ld, steps=2)
    best = th[torch.tensor(wl.cand_off[:-1], device="cuda")].contiguous()
    lb = torch.tensor(wl.lb, device="cuda")
    ub = torch.tensor(wl.ub, device="cuda")
    with pytest.raises(D.DebyeError):
        pol.run(b1, best, lb, ub, flags=D.FLAG_DD_REFINE)
    with pytest.raises(ValueError):
        D.DebyeCost.apply(th.clone().requires_grad_(True), b.eps_re, b.eps_im, plan, b, 1e-8, D.FLAG_DD_REFINE)
    # the flag with the sign flip off is accepted
    D.fit_eval(plan, b, th, flags=D.FLAG_DD_REFINE | D.FLAG_NO_SIGN_FLIP)
    torch.cuda.synchronize()
