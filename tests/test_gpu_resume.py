"""Checkpoint/resume of the batched optimisers on the GPU.

The swarm (Sec. III-A/B) and the DE and DA populations draw their random
numbers from a counter-based generator keyed by (seed, material, iteration,
member, coordinate), so their whole state is the arrays the library updates.
Saving those arrays to a file after K iterations, dropping every GPU object,
and continuing from the file for K more iterations must give the state of an
uninterrupted run of 2K iterations bit for bit.  (The oracle's swarm is
pinned the same way on the CPU.)"""
import numpy as np
import pytest

from _helpers import small_ragged, targets_oracle

pytestmark = pytest.mark.gpu

K = 6


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


@pytest.fixture(scope="module")
def case(orc):
    wl = small_ragged(10, seed=33, Fr=(40, 300), Nr=(2, 20), Pr=(8, 70))
    er, ei = targets_oracle(orc, wl)
    return wl, er, ei


def _batch(D, wl, er, ei):
    return D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, _t(er), _t(ei))


def _save(path, state, t, cost):
    # the iteration and the last evaluation's costs beside the state arrays
    np.savez(path, resume_t=t, resume_cost=cost.cpu().numpy(),
             **{k: v.cpu().numpy() for k, v in vars(state).items()})


def _load(cls, path):
    import torch
    z = np.load(path)   # written by this test; plain arrays, no pickles
    fields = {k: torch.tensor(z[k], device="cuda") for k in z.files if not k.startswith("resume_")}
    return cls(**fields), int(z["resume_t"]), torch.tensor(z["resume_cost"], device="cuda")


def _same(a, b, what):
    for k, v in vars(a).items():
        x, y = v.cpu().numpy(), getattr(b, k).cpu().numpy()
        assert np.array_equal(x, y, equal_nan=True), f"{what}: {k} differs after resume"


def test_pso_resume_is_bit_exact(D, case, tmp_path):
    import torch
    wl, er, ei = case
    lb, ub = _t(wl.lb), _t(wl.ub)

    def run(sw, b, plan, t0, t1, cost):
        for t in range(t0, t1 + 1):
            D.pso_step(b, lb, ub, sw, t, True, cost, wl.inertia, wl.c1, wl.c2, 5)
            cost = D.fit_eval(plan, b, sw.x, want_weights=False)[0]
        return cost

    b = _batch(D, wl, er, ei)
    plan = D.Plan(b)
    ref = D.Swarm.empty(wl.P, wl.M, wl.ld, 2 * K + 2)
    D.pso_init(b, lb, ub, ref, wl.inertia, wl.c1, wl.c2, 5)
    c0 = D.fit_eval(plan, b, ref.x, want_weights=False)[0]
    c_ref = run(ref, b, plan, 1, 2 * K, c0)

    sw = D.Swarm.empty(wl.P, wl.M, wl.ld, 2 * K + 2)
    D.pso_init(b, lb, ub, sw, wl.inertia, wl.c1, wl.c2, 5)
    c = run(sw, b, plan, 1, K, D.fit_eval(plan, b, sw.x, want_weights=False)[0])
    torch.cuda.synchronize()
    _save(tmp_path / "pso.npz", sw, K, c)
    del sw, c, plan, b
    torch.cuda.empty_cache()

    b2 = _batch(D, wl, er, ei)
    plan2 = D.Plan(b2)
    sw2, t, c = _load(D.Swarm, tmp_path / "pso.npz")
    c2 = run(sw2, b2, plan2, t + 1, 2 * K, c)
    torch.cuda.synchronize()
    _same(ref, sw2, "PSO")
    assert torch.equal(c_ref, c2)


@pytest.mark.parametrize("alg", ["de", "da"])
def test_population_resume_is_bit_exact(D, case, tmp_path, alg):
    import torch
    wl, er, ei = case
    lb, ub = _t(wl.lb), _t(wl.ub)
    init, propose, accept = ((D.de_init, D.de_trial, D.de_select) if alg == "de" else
                             (D.da_init, D.da_visit, D.da_accept))

    def step(pop, b, plan, t):
        propose(b, lb, ub, pop, t, seed=9)
        cost = D.fit_eval(plan, b, pop.u, want_weights=False)[0]
        if alg == "de":
            accept(b, pop, t, pop.u, cost)
        else:
            accept(b, pop, t, pop.u, cost, seed=9)
        return cost

    def start(b, plan):
        pop = D.Population.empty(wl.P, wl.M, wl.ld, 2 * K + 2)
        init(b, lb, ub, pop, seed=9)
        cost = D.fit_eval(plan, b, pop.x, want_weights=False)[0]
        if alg == "de":
            accept(b, pop, 0, pop.x, cost)
        else:
            accept(b, pop, 0, pop.x, cost, seed=9)
        return pop, cost

    b = _batch(D, wl, er, ei)
    plan = D.Plan(b)
    ref, c = start(b, plan)
    for t in range(1, 2 * K + 1):
        c = step(ref, b, plan, t)

    pop, c = start(b, plan)
    for t in range(1, K + 1):
        c = step(pop, b, plan, t)
    torch.cuda.synchronize()
    _save(tmp_path / f"{alg}.npz", pop, K, c)
    del pop, plan, b
    torch.cuda.empty_cache()

    b2 = _batch(D, wl, er, ei)
    plan2 = D.Plan(b2)
    pop2, t0, _ = _load(D.Population, tmp_path / f"{alg}.npz")
    for t in range(t0 + 1, 2 * K + 1):
        step(pop2, b2, plan2, t)
    torch.cuda.synchronize()
    _same(ref, pop2, alg.upper())
