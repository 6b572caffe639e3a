"""The persistent launch of a ragged evaluation (one kernel over every
pole-count bucket, work items taken per XCD from a counter in device memory)
against the per-bucket launches and the oracle."""
import numpy as np
import pytest

import workloads as W
from _helpers import COST_RTOL, attributed_cost_err, cost_floor, cost_rel_err, small_ragged, targets_oracle

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


@pytest.mark.parametrize("seed,split", [(41, None), (42, "tune"), (43, 1), (44, 8)])
def test_persistent_launch_equals_bucket_launches(D, orc, seed, split):
    """Every pole count 1..24, uneven spectra and swarm sizes (some empty):
    the persistent launch gives the per-bucket launches' results bit for bit,
    and both match the oracle."""
    import torch
    wl = small_ragged(48, seed=seed, Fr=(20, 600), Nr=(1, 24), Pr=(0, 90))
    er, ei = targets_oracle(orc, wl)
    b = D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, _t(er), _t(ei))
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=seed)
    th = _t(theta)
    plan = D.Plan(b)
    if split == "tune":
        plan.autotune(b, th, reps=1)
    elif split:
        plan.set_freq_split(split)
    print(f"[persistent {seed}] {len(plan.info())} buckets, schedule {plan.info()}, autotuned mode {plan.launch()}",
          flush=True)
    plan.set_launch(D.LAUNCH_BUCKETS)
    ref = D.fit_eval(plan, b, th)
    torch.cuda.synchronize()
    plan.set_launch(D.LAUNCH_PERSISTENT)
    assert plan.launch() == D.LAUNCH_PERSISTENT
    got = D.fit_eval(plan, b, th)
    torch.cuda.synchronize()
    # weights: only the first n_poles entries of a row are written
    npc = torch.tensor(np.repeat(wl.n_poles, np.diff(wl.cand_off)), device="cuda")
    used = torch.arange(wl.ld, device="cuda")[None, :] < npc[:, None]
    for name, x, y in zip(("cost", "weights", "eps_inf", "status"), ref, got):
        if name == "weights":
            x, y = x[used], y[used]
        assert torch.equal(torch.nan_to_num(x.float() if x.dtype == torch.int8 else x, nan=7.25),
                           torch.nan_to_num(y.float() if y.dtype == torch.int8 else y, nan=7.25)), name
    ob = orc.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, er, ei)
    oc, _, _, ost = orc.fit_eval(ob, theta)
    np.testing.assert_array_equal(got[3].cpu().numpy(), ost)
    c = got[0].cpu().numpy()
    floor = cost_floor(wl, er, ei)
    rel, _ = attributed_cost_err(orc, ob, theta, c, floor, 1e-8, 0, cost_rel_err(c, oc, floor))
    print(f"[persistent {seed}] max cost rel err {rel.max():.2e} over {wl.P} candidates", flush=True)
    assert rel.max() <= COST_RTOL


def test_persistent_launch_in_the_swarm_graph(D, orc):
    """A whole swarm fit replayed from its captured graph with the persistent
    launch equals the eager fit, and the fit with per-bucket launches."""
    import torch
    wl = small_ragged(24, seed=45, Fr=(30, 300), Nr=(2, 20), Pr=(8, 64))
    wl.iters = 6
    er, ei = targets_oracle(orc, wl)
    b = D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, _t(er), _t(ei))
    lb, ub = _t(wl.lb), _t(wl.ub)
    out = {}
    for mode, graph in ((D.LAUNCH_BUCKETS, False), (D.LAUNCH_PERSISTENT, False), (D.LAUNCH_PERSISTENT, True)):
        plan = D.Plan(b)
        plan.set_launch(mode)
        sw = D.Swarm.empty(wl.P, wl.M, wl.ld, wl.iters + 1)
        D.pso_run(plan, b, lb, ub, sw, wl.iters, seed=3, use_graph=graph)
        torch.cuda.synchronize()
        out[(mode, graph)] = (sw.gbest_cost.clone(), sw.gbest_x.clone(), sw.x.clone())
    base = out[(D.LAUNCH_BUCKETS, False)]
    for k, v in out.items():
        for x, y in zip(base, v):
            assert torch.equal(x, y), k
