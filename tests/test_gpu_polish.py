"""GPU checks of the L-BFGS polish context (debye_polish_*): its history
handling against the oracle when curvature pairs are rejected with a full
history, one step captured into a HIP graph and replayed bit for bit against
eager steps, and the zeroed padding of the theta-gradient rows."""
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


def test_polish_rejected_pairs_keep_history(D, orc):
    """Polish from random starts with memory 1: many accepted steps have
    s.y <= 1e-300 (steps clamped at the box) while the history is full, and
    their pairs must not replace the live one.  The GPU cost history follows
    the oracle's at every step on the materials where such a rejection happens
    (those with a perturbation-stable oracle trajectory)."""
    import torch
    wl = W.hn_cc(M=256, F=200, N=2, P=1, iters=0, seed=1)
    er, ei = targets_oracle(orc, wl)
    one = np.arange(wl.M + 1)
    th0 = W.draw_theta(one, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=11)
    ob = orc.Batch(wl.f_off, one, wl.n_poles, wl.omega, er, ei)
    steps = 25
    oth, ohist, rej = orc.lbfgs(ob, th0, wl.lb, wl.ub, steps=steps, mem=1, rejected=True)
    # materials whose oracle trajectory is stable: starts moved by 1e-14
    # (relative) leave their cost history within 1e-9 (elsewhere near-tied
    # line-search decisions make any two FP64 runs part ways)
    stable = np.ones(wl.M, bool)
    for eps in (1e-14, -1e-14):
        _, h = orc.lbfgs(ob, th0 * (1 + eps), wl.lb, wl.ub, steps=steps, mem=1)
        stable &= np.max(np.abs(h - ohist) / ohist, axis=1) <= 1e-9
    sel = np.nonzero((rej > 0) & stable)[0]
    assert len(sel) >= 20
    b1 = D.Batch(wl.f_off, one, wl.n_poles, wl.omega, _t(er), _t(ei))
    th = _t(th0)
    hist = D.lbfgs_polish(b1, th, _t(wl.lb), _t(wl.ub), steps=steps, mem=1).cpu().numpy()
    torch.cuda.synchronize()
    err = np.max(np.abs(hist[sel] - ohist[sel]) / ohist[sel], axis=1)
    print(f"[polish rejected pairs] {len(sel)} materials, max rel history diff {err.max():.2e}", flush=True)
    assert np.all(np.diff(hist, axis=1) <= 0)
    assert np.all(err <= 1e-6), sel[err > 1e-6]


def test_polish_step_graph_replay_is_bit_identical(D, orc):
    """One polish step captured into a HIP graph (the context allocates and
    synchronises nothing) and replayed six times, with eager work and
    synchronisations between the replays, equals six eager steps bit for bit
    after every replay."""
    import torch
    wl = W.hn_cc(M=40, F=300, N=8, P=1, iters=0, seed=3)
    er, ei = targets_oracle(orc, wl)
    one = np.arange(wl.M + 1)
    th0 = W.draw_theta(one, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=4)
    b1 = D.Batch(wl.f_off, one, wl.n_poles, wl.omega, _t(er), _t(ei))
    lb, ub = _t(wl.lb), _t(wl.ub)
    K = 6
    # eager
    pe = D.Polish(b1, wl.ld, steps=K)
    the = _t(th0)
    pe.begin(b1, the)
    eager = []
    for k in range(K):
        pe.step(b1, the, lb, ub, k)
        eager.append(the.clone())
    torch.cuda.synchronize()
    # captured
    pg = D.Polish(b1, wl.ld, steps=K)
    thg = _t(th0)
    pg.begin(b1, thg)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            pg.step(b1, thg, lb, ub, 0)
    torch.cuda.synchronize()
    # capture does not run the step
    np.testing.assert_array_equal(thg.cpu().numpy(), th0)
    other = D.Batch(wl.f_off, one, wl.n_poles, wl.omega, _t(er), _t(ei))
    plan_o = D.Plan(other)
    for k in range(K):
        g.replay()
        torch.cuda.synchronize()
        D.fit_eval(plan_o, other, _t(th0), want_weights=False)
        torch.cuda.synchronize()
        assert torch.equal(thg, eager[k]), f"replay {k}"
    assert not torch.equal(eager[-1], _t(th0))


def test_theta_gradient_padding_is_zero(D, orc):
    """Ragged pole counts in rows of stride ld > N_m: the adjoint writes 0 into
    the padding entries, so DebyeCost's theta.grad is exactly 0 there."""
    import torch
    wl = small_ragged(10, seed=77, Fr=(40, 200), Nr=(2, 12), Pr=(3, 20))
    er, ei = targets_oracle(orc, wl)
    b = D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, _t(er), _t(ei))
    plan = D.Plan(b)
    th = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=2)
    th = np.where(np.isnan(th), -9.0, th)      # padding holds ordinary numbers
    theta = _t(th).requires_grad_(True)
    # poison the memory the gradient will be allocated from
    junk = torch.full((wl.P * wl.ld * 4,), float("nan"), dtype=torch.float64, device="cuda")
    del junk
    cost = D.DebyeCost.apply(theta, _t(er), _t(ei), plan, b)
    cost.sum().backward()
    g = theta.grad.cpu().numpy()
    npc = np.repeat(wl.n_poles, np.diff(wl.cand_off))
    assert np.any(npc < wl.ld)
    for c in range(wl.P):
        assert np.all(g[c, npc[c]:] == 0.0), c
        assert np.all(np.isfinite(g[c, :npc[c]]))
