"""Every workload at its full size, in the launch configuration the bench
times (one plan over the whole batch, autotuned schedule): one evaluation of
all candidates on the GPU, a sample of them checked one by one against the
oracle (targets included), and for the HN/CC workload the adjoint too."""
import numpy as np
import pytest

import workloads as W
from _helpers import COST_RTOL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    import paper_2109_01928_amd as D

    assert torch.cuda.is_available()
    D.lib()
    return D


def _sample_batch(orc, wl, mats):
    """Oracle batch of the sampled candidates' materials (one candidate each),
    targets from the oracle with each material's own noise stream."""
    F = np.diff(wl.f_off)[mats]
    fo = np.concatenate([[0], np.cumsum(F)])
    om = np.concatenate([wl.omega[wl.f_off[m]:wl.f_off[m + 1]] for m in mats])
    er, ei = orc.material_eval_sample(wl.kind[mats], wl.params[mats], fo, om, mats, noise_seed=wl.noise_seed)
    return orc.Batch(fo, np.arange(len(mats) + 1), wl.n_poles[mats], om, er, ei), er, ei


def _gpu_full(D, wl):
    import torch
    z = np.zeros(len(wl.omega))
    b0 = D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, z, z)
    er, ei = D.material_eval(wl.kind, wl.params, b0, noise_seed=wl.noise_seed)
    b = b0.with_targets(er, ei)
    theta = torch.tensor(W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=91), device="cuda")
    plan = D.Plan(b)
    plan.autotune(b, theta, reps=1)
    return b, er, ei, theta, plan


def _judge(orc, sub, th, c_gpu, er, ei, n):
    oc = orc.fit_eval(sub, th)[0]
    per = np.array([np.sum(er[sub.f_off[i]:sub.f_off[i + 1]] ** 2 + ei[sub.f_off[i]:sub.f_off[i + 1]] ** 2)
                    for i in range(n)])
    floor = 1e-12 * per
    stats = {}
    rel, _ = orc.judge_costs(sub, th, c_gpu, oc, floor, COST_RTOL, stats=stats)
    return rel, stats


@pytest.mark.parametrize("which,sample", [("ragged", 1024), ("tables", 192)])
def test_full_size_forward(D, orc, which, sample):
    import torch
    wl = W.mixed_ragged(M=4096, iters=1) if which == "ragged" else W.tables(M=65536, iters=1)
    b, er, ei, theta, plan = _gpu_full(D, wl)
    c, _, _, st = D.fit_eval(plan, b, theta, want_weights=False)
    torch.cuda.synchronize()
    print(f"{which}: {wl.P} candidates in one evaluation, schedule {plan.info()}", flush=True)
    rng = np.random.default_rng(2)
    idx = np.sort(rng.choice(wl.P, sample, replace=False))
    mats = np.searchsorted(wl.cand_off, idx, side="right") - 1
    sub, oer, oei = _sample_batch(orc, wl, mats)
    # GPU targets of the sampled materials against the oracle's
    ger = np.concatenate([er[wl.f_off[m]:wl.f_off[m + 1]].cpu().numpy() for m in mats])
    gei = np.concatenate([ei[wl.f_off[m]:wl.f_off[m + 1]].cpu().numpy() for m in mats])
    assert np.max(np.abs(ger - oer) / np.abs(oer)) < 1e-12 and np.max(np.abs(gei - oei) / np.abs(oei)) < 1e-12
    th = theta[torch.tensor(idx, device="cuda")].cpu().numpy()
    cg = c.cpu().numpy()[idx]
    assert np.all(st.cpu().numpy()[idx] == 0)
    rel, stats = _judge(orc, sub, th, cg, oer, oei, len(idx))
    print(f"{which} full-size sample: {stats}, max rel err {rel.max():.3e}", flush=True)
    assert rel.max() <= COST_RTOL


def test_full_size_hn_cc_forward_and_adjoint(D, orc):
    import torch
    wl = W.hn_cc(M=1024, iters=1)
    b, er, ei, theta, plan = _gpu_full(D, wl)
    c, g, _, _, st = D.fit_eval_grad(plan, b, theta)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    idx = np.sort(rng.choice(wl.P, 256, replace=False))
    mats = idx // 256
    sub, oer, oei = _sample_batch(orc, wl, mats)
    th = theta[torch.tensor(idx, device="cuda")].cpu().numpy()
    rel, stats = _judge(orc, sub, th, c.cpu().numpy()[idx], oer, oei, len(idx))
    print(f"hn-cc full-size sample: {stats}, max rel err {rel.max():.3e}", flush=True)
    assert rel.max() <= COST_RTOL
    oc, og, _, _, ost = orc.fit_grad(sub, th)
    gg = g.cpu().numpy()[idx]
    gerr = np.max(np.abs(gg[:, :12] - og[:, :12]), axis=1) / np.max(np.abs(og[:, :12]), axis=1)
    print(f"hn-cc full-size sample: max theta-gradient rel err {gerr.max():.2e}", flush=True)
    assert np.all(gerr <= 1e-6)


def test_spectrum_past_32bit_offsets(D, orc):
    """One material whose spectrum holds more than 2^29 points (past the
    uniform tile form's 32-bit byte offsets, so the plan takes the general form
    with 64-bit point indices).  The spectrum repeats a 1,000-point one K times,
    which multiplies every frequency sum by K: the weights, eps_inf and status
    are those of the short spectrum, and the cost and its adjoint K times
    theirs (the oracle on the short spectrum).  Tolerances: a lane sums
    n = F / split points in order, so its sums carry relative errors up to
    about n u (u = 2^-53); the weights that times the condition number of the
    equilibrated damped Gram matrix; the adjoint the parity tests' 1e-6."""
    import torch
    wl = W.mixed_uniform(M=1, F=1000, N=2, P=8, iters=1, seed=13)
    er, ei = orc.material_eval(wl.kind, wl.params, wl.f_off, wl.omega, noise_seed=wl.noise_seed)
    F0 = len(wl.omega)
    K = (1 << 29) // F0 + 1
    F = K * F0
    lo = float(wl.lb[0])
    theta = np.array([[lo + 0.3 + 0.3 * i, lo + 2.3 + 0.3 * i] for i in range(8)])   # poles 2 decades apart
    assert np.all(theta <= wl.ub[0])
    print(f"[long spectrum] F = {F} ({K} x {F0})", flush=True)
    big = [torch.tensor(a, device="cuda").repeat(K) for a in (wl.omega, er, ei)]
    b = D.Batch(np.array([0, F]), wl.cand_off, wl.n_poles, big[0], big[1], big[2])
    plan = D.Plan(b)
    info = plan.info()
    assert len(info) == 1 and not info[0]["uniform"], info
    split = info[0]["freq_split"]
    th = torch.tensor(theta, device="cuda")
    c, w, einf, st = D.fit_eval(plan, b, th)
    c_dd = D.fit_eval(plan, b, th, flags=D.FLAG_DD_REFINE, want_weights=False)[0]
    cg, g, _, _, stg = D.fit_eval_grad(plan, b, th)
    torch.cuda.synchronize()
    c, w, einf, st, c_dd, cg, g, stg = (x.cpu().numpy() for x in (c, w, einf, st, c_dd, cg, g, stg))
    del big, b, plan
    torch.cuda.empty_cache()

    ob = orc.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, er, ei)
    oc, ow, oe, ost = orc.fit_eval(ob, theta)
    _, og = orc.fit_grad(ob, theta)[:2]
    np.testing.assert_array_equal(st, ost)
    np.testing.assert_array_equal(stg, ost)
    assert np.all(ost == 0)
    n_sum = -(-F // split) + 64
    u = 2.0 ** -53
    lam = 1e-8
    kappa = 0.0
    for t in theta:
        x = wl.omega[:, None] * 10.0 ** t[None, :]
        I = x / (1.0 + x * x)
        Mg = I.T @ I
        Mg = Mg + lam * np.diag(np.diag(Mg))
        d = 1.0 / np.sqrt(np.diag(Mg))
        kappa = max(kappa, np.linalg.cond(Mg * d[:, None] * d[None, :]))
    rel_c = np.abs(c - K * oc) / (K * oc)
    rel_dd = np.abs(c_dd - K * oc) / (K * oc)
    rel_w = np.max(np.abs(w - ow)) / np.max(np.abs(ow))
    rel_e = np.max(np.abs(einf - oe) / np.abs(oe))
    rel_g = np.max(np.abs(g - K * og), axis=1) / np.max(np.abs(K * og), axis=1)
    print(f"[long spectrum] split {split}, {n_sum} terms per lane, kappa {kappa:.1f}: cost {rel_c.max():.2e} "
          f"(dd {rel_dd.max():.2e}), weights {rel_w:.2e}, eps_inf {rel_e:.2e}, adjoint {rel_g.max():.2e}", flush=True)
    assert np.max(np.abs(cg - K * oc) / (K * oc)) <= 8 * n_sum * u
    assert rel_c.max() <= 8 * n_sum * u
    assert rel_dd.max() <= 8 * n_sum * u
    assert rel_w <= 8 * kappa * n_sum * u
    assert rel_e <= 8 * kappa * n_sum * u
    assert rel_g.max() <= 1e-6
