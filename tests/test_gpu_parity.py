"""GPU parity of the HIP library against the FP64 oracle, called through the C
ABI (via the thin binding).  Same seeded inputs on both sides; targets are
computed by the oracle and uploaded, so the cost kernels see identical data."""
import json
import os
import sys

import numpy as np
import pytest

import workloads as W
from _helpers import (COST_RTOL, WEIGHT_RTOL, attributed_cost_err, attributed_weight_err, cost_floor, cost_rel_err,
                      weight_rel_err,
                      mixed_scale_workload, poles_per_cand, small_ragged, small_uniform, targets_oracle)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    import paper_2109_01928_amd as D

    assert torch.cuda.is_available()
    D.lib()
    return D


def _gpu_batch(D, wl, er, ei):
    import torch
    return D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, torch.tensor(er, device="cuda"),
                   torch.tensor(ei, device="cuda"))


def _domain_split(orc, ob, theta, c_gpu, ost, edge, damping, flags, floor, tag):
    """Candidates at the edge of the admissible domain (poles many decades
    outside the band): status parity is asserted for all of them; cost parity
    only where the cost is determined by FP64 arithmetic to well within the
    tolerance (cond * u <= 1e-11, cond from the oracle's sensitivity measure).
    The rest are counted, with the GPU's, the FP64 oracle's and the 80-bit
    oracle's errors against the binary128 oracle printed.  Returns the mask
    of candidates whose cost parity is asserted."""
    assert_mask = np.ones(len(c_gpu), bool)
    if not edge:
        return assert_mask
    idx = np.array(sorted(edge))
    cond = orc.fit_cond_batch(ob, theta, damping, flags)[idx]
    ok = ost[idx] == 0
    determined = ok & (cond * orc.UNIT_ROUNDOFF <= 1e-11)
    assert_mask[idx[~determined]] = False
    rest = idx[~determined & ok]
    if len(rest):
        c128 = orc.fit_eval(ob, theta, damping, flags, precision=128)[0][rest]
        c64 = orc.fit_eval(ob, theta, damping, flags)[0][rest]
        c80 = orc.fit_eval(ob, theta, damping, flags, precision=80)[0][rest]
        den = np.maximum(c128, floor[rest])
        e = lambda c: np.abs(c - c128) / den
        print(f"[{tag}] {len(rest)} edge candidates with cond*u > 1e-11 (not asserted); errors vs binary128: "
              f"GPU max {e(c_gpu[rest]).max():.2e}, FP64 oracle max {e(c64).max():.2e}, "
              f"80-bit oracle max {e(c80).max():.2e}", flush=True)
    return assert_mask


def _check_eval(D, orc, wl, theta, damping=1e-8, flags=0, split=None, tag="", edge=(), gpu_flags=0):
    """The GPU evaluation under flags | gpu_flags (gpu_flags: flags that change
    only how accurately the same result is computed) against the oracle's
    under flags."""
    import torch
    er, ei = targets_oracle(orc, wl)
    ob = orc.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, er, ei)
    oc, ow, oe, ost = orc.fit_eval(ob, theta, damping=damping, flags=flags)
    b = _gpu_batch(D, wl, er, ei)
    plan = D.Plan(b)
    th = torch.tensor(theta, device="cuda")
    if split == "tune":
        plan.autotune(b, th, damping=damping, flags=flags | gpu_flags, reps=1)
    elif split:
        plan.set_freq_split(split)
    c, w, e, st = D.fit_eval(plan, b, th, damping=damping, flags=flags | gpu_flags)
    torch.cuda.synchronize()
    c, w, e, st = (t.cpu().numpy() for t in (c, w, e, st))
    print(f"[{tag}] {wl.name} split={split} plan={plan.info()}", flush=True)
    np.testing.assert_array_equal(st, ost)
    floor = cost_floor(wl, er, ei)
    sel = _domain_split(orc, ob, theta, c, ost, edge, damping, flags, floor, tag)
    rel, n_lim = attributed_cost_err(orc, ob, theta[sel], c[sel], floor[sel], damping, flags,
                                     cost_rel_err(c, oc, floor)[sel]) if sel.all() else \
        _judge_subset(orc, ob, theta, c, floor, damping, flags, oc, sel)
    worst = int(np.argmax(rel))
    print(f"[{tag}] max cost rel err {rel.max():.3e}; oracle-limited candidates: {n_lim} of {int(sel.sum())}",
          flush=True)
    assert rel.max() <= COST_RTOL, f"cost rel err {rel.max():.3e} at candidate {worst}"
    ok = (ost == 0) & sel
    if edge:
        # the weights of an edge candidate can be far more sensitive than its
        # cost: asserted where the FP64 and 80-bit oracles' weights both agree
        # with the binary128 oracle's within WEIGHT_RTOL / 10, counted otherwise
        idx = np.nonzero(ok)[0]
        idx = idx[np.isin(idx, np.array(sorted(edge)))]
        npc = poles_per_cand(wl)
        w128 = orc.fit_eval(ob, theta, damping, flags, precision=128)[1]
        w80 = orc.fit_eval(ob, theta, damping, flags, precision=80)[1]
        det = (weight_rel_err(ow[idx], w128[idx], npc[idx]) <= WEIGHT_RTOL / 10) & \
              (weight_rel_err(w80[idx], w128[idx], npc[idx]) <= WEIGHT_RTOL / 10)
        ok[idx[~det]] = False
        print(f"[{tag}] weights of {int((~det).sum())} edge candidates not determined to {WEIGHT_RTOL / 10:g} by "
              f"FP64 or 80-bit arithmetic (not asserted)", flush=True)
    werr, eerr, n_wlim = attributed_weight_err(orc, ob, theta, w, e, ok, poles_per_cand(wl), damping, flags, ow, oe)
    print(f"[{tag}] max weight rel err {werr.max(initial=0):.3e}, eps_inf {eerr.max(initial=0):.3e}; "
          f"oracle-limited: {n_wlim}", flush=True)
    assert werr.max(initial=0) <= WEIGHT_RTOL, f"weight rel err {werr.max():.3e}"
    assert eerr.max(initial=0) <= WEIGHT_RTOL, f"eps_inf rel err {eerr.max():.3e}"
    return rel.max(), werr.max(initial=0)


def _judge_subset(orc, ob, theta, c, floor, damping, flags, oc, sel):
    """attributed_cost_err over the candidates in `sel` (errors of the others 0)."""
    rel = np.zeros(len(c))
    r64 = cost_rel_err(c, oc, floor)
    over = np.nonzero(sel & ~(r64 <= COST_RTOL))[0]
    rel[sel] = r64[sel]
    n = 0
    for i in over:
        m = int(np.searchsorted(ob.cand_off, i, side="right") - 1)
        f0, f1 = ob.f_off[m], ob.f_off[m + 1]
        one = orc.Batch([0, f1 - f0], [0, 1], ob.n_poles[m:m + 1], ob.omega[f0:f1], ob.eps_re[f0:f1],
                        ob.eps_im[f0:f1])
        r, k = attributed_cost_err(orc, one, theta[i:i + 1], c[i:i + 1], floor[i:i + 1], damping, flags,
                                   r64[i:i + 1])
        rel[i] = r[0]
        n += k
    return rel, n


# ---------------------------------------------------------------------------
def test_material_targets_match_oracle(D, orc):
    import torch
    for wl in (small_uniform(40, 333, 5, 1, seed=4), small_ragged(30, seed=2), W.tables(M=16, F=257, N=20, P=1)):
        er, ei = targets_oracle(orc, wl)
        b = D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, np.zeros_like(er), np.zeros_like(er))
        ger, gei = D.material_eval(wl.kind, wl.params, b, noise_seed=wl.noise_seed)
        torch.cuda.synchronize()
        np.testing.assert_allclose(ger.cpu().numpy(), er, rtol=2e-13, atol=1e-13)
        np.testing.assert_allclose(gei.cpu().numpy(), ei, rtol=2e-13, atol=1e-13)
    # Jacobian of the HN family
    wl = small_uniform(24, 101, 5, 1, seed=8, kinds=[W.KIND_HN, W.KIND_CC, W.KIND_CD])
    oer, oei, oJ = orc.material_eval(wl.kind, wl.params, wl.f_off, wl.omega, jac=True)
    b = D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, oer, oei)
    ger, gei, gJ = D.material_eval(wl.kind, wl.params, b, jac=True)
    gJ = gJ.cpu().numpy()
    scale = np.abs(oJ).max(axis=(0, 2))                       # per parameter column
    assert np.max(np.abs(gJ - oJ).max(axis=(0, 2)) / scale) < 1e-12


def test_basis_matches_oracle(D, orc):
    import torch
    om = W.log_grid(1e5, 1e11, 777)
    theta = np.array([[-12.5, -11.0, -9.3, -7.7, -6.2], [-10.0, -10.0, -8.0, -7.0, -9.9]])
    re, im = D.basis(torch.tensor(om, device="cuda"), torch.tensor(theta, device="cuda"), 5)
    for c in range(2):
        r0, i0 = orc.basis(om, theta[c])
        np.testing.assert_allclose(re[c].cpu().numpy(), r0, rtol=1e-15, atol=0)
        np.testing.assert_allclose(im[c].cpu().numpy(), i0, rtol=1e-15, atol=0)


def test_listing2_on_gpu(D, orc):
    import torch
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "listing2.json")))
    m = g["material"]
    om = W.log_grid(1e7, 1e11, 100)
    p = np.zeros((1, 16))
    p[0, :5] = [m["eps_inf"], m["d_eps"], m["tau0"], m["alpha"], m["beta"]]
    b = D.Batch([0, 100], [0, 1], [5], om, np.zeros(100), np.zeros(100))
    er, ei = D.material_eval([W.KIND_HN], p, b)
    b = b.with_targets(er, ei)
    th = torch.tensor(np.log10(g["printed_tau"])[None], device="cuda")
    for damping in (0.0, 1e-8):
        c, w, e, st = D.fit_eval(D.Plan(b), b, th, damping=damping)
        assert st.item() == 0
        np.testing.assert_array_equal(np.round(w.cpu().numpy()[0], 4), g["printed_d_eps"])
        assert round(e.item(), 4) == g["printed_eps_inf"]


# cost parity at the shapes of the benchmark workloads (reduced counts), every
# pole-count branch and every frequency split
@pytest.mark.parametrize("F,N,P,M,fmin,fmax", [
    (50, 5, 40, 1, 1e5, 1e10),        # single HN workload shape
    (1000, 8, 64, 6, 1e6, 1e10),      # mixed batch shape (bench workload)
    (2000, 12, 32, 4, 1e5, 1e11),     # differentiation workload shape
    (4096, 20, 16, 2, 1e5, 1e11),     # tables workload shape
])
def test_cost_parity_config_shapes(D, orc, F, N, P, M, fmin, fmax):
    wl = small_uniform(M, F, N, P, seed=F + N, fmin=fmin, fmax=fmax)
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=N)
    r, wr = _check_eval(D, orc, wl, theta, tag="shape")
    print(f"F={F} N={N}: max cost rel err {r:.2e}, weights {wr:.2e}")


@pytest.mark.parametrize("N", list(range(1, 25)))
def test_cost_parity_every_pole_count(D, orc, N):
    wl = small_uniform(3, 173, N, 70, seed=100 + N)   # 70 candidates: ragged last tile
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=N)
    sp = D.Plan(_gpu_batch(D, wl, *targets_oracle(orc, wl))).info()[0]["pole_split"]
    for split in (None, 1, 4, 64 // sp):
        _check_eval(D, orc, wl, theta, split=split, tag=f"N{N}")


@pytest.mark.parametrize("N", list(range(1, 25)))
def test_dd_refine_parity_every_pole_count(D, orc, N):
    """DEBYE_FLAG_DD_REFINE on the same batches (its kernels take the general
    tile form for every tile), at the automatic and the widest split."""
    wl = small_uniform(3, 173, N, 70, seed=100 + N)
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=N)
    sp = D.Plan(_gpu_batch(D, wl, *targets_oracle(orc, wl))).info()[0]["pole_split"]
    for split in (None, 64 // sp):
        _check_eval(D, orc, wl, theta, split=split, tag=f"dd N{N}", gpu_flags=D.FLAG_DD_REFINE)


@pytest.mark.parametrize("N", [8, 12, 20])
def test_dd_refine_parity_extreme_relaxation_times(D, orc, N):
    """The double-double basis at the ends of the admissible range: poles
    spread over 60 decades, w tau up to 6e19, poles far above the band."""
    wl = small_uniform(2, 200, N, 64, seed=40 + N)
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=N)
    theta[3, :N] = np.linspace(-30.0, 30.0, N)
    theta[70, :N] = np.linspace(6.0, 9.0, N)
    theta[71, :N] = np.linspace(-29.0, -26.0, N)
    _check_eval(D, orc, wl, theta, tag=f"dd extreme N{N}", edge=(3, 70, 71), gpu_flags=D.FLAG_DD_REFINE)


@pytest.mark.parametrize("N", [12, 17, 20, 24])
def test_cost_parity_short_spectra(D, orc, N):
    """Spectra shorter than a candidate's lanes (F from 1 to 21 at frequency
    splits up to 64 / SP): lanes and point subsets with no points, the
    refinement pass's tails of one to three points, and fewer points than
    poles (the damped system stays definite)."""
    Fm = [1, 2, 3, 5, 8, 13, 21]
    M = len(Fm)
    kind, params = W.draw_mixed(M, 500 + N, 1e6, 1e10)
    lb, ub = W.tau_bounds(1e6, 1e10)
    om = np.concatenate([W.log_grid(1e6, 1e10, f) for f in Fm])
    wl = W.Workload(f"short spectra N{N}", kind, params, W.offsets(Fm), om, np.full(M, N, np.int32),
                    W.offsets([24] * M), np.full(M, lb), np.full(M, ub), 1, seed=500 + N)
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=N)
    sp = D.Plan(_gpu_batch(D, wl, *targets_oracle(orc, wl))).info()[0]["pole_split"]
    for split in sorted({1, 2, 8, 64 // sp}):
        _check_eval(D, orc, wl, theta, split=split, tag=f"short N{N}")


@pytest.mark.parametrize("N", [6, 12, 20])
def test_cost_parity_uniform_and_mixed_tiles(D, orc, N):
    """Both tile forms at split 1 and wider splits: whole swarms of 64 (every
    wave one material: wave-uniform spectrum addresses) and swarms of 12
    (waves shared by two materials)."""
    seen = set()
    for P, M in ((64, 4), (12, 16)):
        wl = small_uniform(M, 211, N, P, seed=300 + N + P)
        theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=N + P)
        er, ei = targets_oracle(orc, wl)
        for split in (1, 2, 4):
            plan = D.Plan(_gpu_batch(D, wl, er, ei))
            plan.set_freq_split(split)
            uni = plan.info()[0]["uniform"]
            # whole waves of 64 are always uniform; 12 per material is where a
            # wave's slots divide 12
            assert uni or P != 64, plan.info()
            seen.add((uni, split == 1))
            _check_eval(D, orc, wl, theta, split=split, tag=f"N{N} P{P} split{split} uniform={uni}")
            del plan
    assert seen == {(True, True), (True, False), (False, True), (False, False)}


@pytest.mark.parametrize("N", [8, 12])
def test_cost_parity_extreme_relaxation_times(D, orc, N):
    """Valid but extreme log10(tau): poles spread over 60 decades (the cost
    pass's scaled coefficients would be subnormal) and poles far below the
    band (w tau up to 1e19: Q(w^2) overflows), beside ordinary candidates in
    the same waves; those waves take the basis form of the cost pass."""
    wl = small_uniform(2, 200, N, 64, seed=40 + N)
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=N)
    theta[3, :N] = np.linspace(-30.0, 30.0, N)               # 60 decades in one candidate
    theta[70, :N] = np.linspace(6.0, 9.0, N)                 # w tau from 6e11 to 6e19
    theta[71, :N] = np.linspace(-29.0, -26.0, N)             # far above the band
    _check_eval(D, orc, wl, theta, tag=f"extreme N{N}", edge=(3, 70, 71))


@pytest.mark.parametrize("N", [3, 8, 13, 20])
def test_cost_parity_full_admissible_range(D, orc, N):
    """Candidates drawn uniformly over the whole admissible range, |log10 tau|
    <= 30 (poles up to 20 decades outside the band), with a few rejected ones
    (|log10 tau| > 30) among them: status parity everywhere; cost parity where
    the cost is determined by FP64 arithmetic to well within the tolerance;
    the rest counted (see _domain_split)."""
    wl = small_uniform(2, 150, N, 48, seed=90 + N)
    theta = np.random.default_rng(N).uniform(-30.0, 30.0, (wl.P, N))
    theta[[5, 50], 0] = [30.5, -31.0]
    _check_eval(D, orc, wl, theta, tag=f"full range N{N}", edge=tuple(range(wl.P)))


@pytest.mark.parametrize("N", [4, 8, 13, 20])
def test_cost_parity_scaled_pole_groups(D, orc, N):
    """The frequency passes share one reciprocal among four poles, on factors
    1 + (w tau)^2 scaled per group by a power of two fixed from the largest
    admissible frequency.  The same HN-family spectra and candidates on the
    ordinary band, on the band moved down by 33 decades (tau near 1e22..1e26:
    every group scaled by about 2^-200) and moved up by 18 decades (w up to
    6e28 rad/s, tau near 1e-29: no group scaled); on each, a rejected
    candidate sets its wave's scale to the cap, 2^-253."""
    import dataclasses
    base = small_uniform(2, 150, N, 64, seed=70 + N, kinds=[W.KIND_HN, W.KIND_CC, W.KIND_CD])
    theta0 = W.draw_theta(base.cand_off, base.n_poles, base.lb, base.ub, base.ld, seed=N)
    for shift in (0, -33, 18):
        params = base.params.copy()
        params[:, 2] *= 10.0 ** -shift          # tau0 of the HN family
        wl = dataclasses.replace(base, name=f"{base.name} band x1e{shift}", params=params,
                                 omega=base.omega * 10.0 ** shift, lb=base.lb - shift, ub=base.ub - shift)
        theta = theta0.copy()
        theta[:, :N] -= shift
        # one rejected candidate (|log10 tau| > 30) among valid ones: its group
        # scale is capped at 2^-253, and the wave's valid lanes then work far
        # below their own scale (their reciprocals near 2^1012)
        theta[5, :N] = 100.0
        _check_eval(D, orc, wl, theta, tag=f"groups N{N} band x1e{shift}")

@pytest.mark.parametrize("N", [4, 5, 8, 9, 12, 13, 16, 17, 20, 24])
def test_cost_parity_mixed_scale_waves(D, orc, N):
    """Two materials with the same HN-family spectrum shape, one on the
    ordinary band and one on the band moved down by 33 decades (tau near
    1e22..1e26, group scales near 2^-200), with 37 candidates each, so that
    tiles mix the two: the ordinary lanes run at the other material's scale,
    far below their own.  Every candidate is in band (well posed), so weights
    are compared too."""
    wl = mixed_scale_workload(N)
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=N)
    _check_eval(D, orc, wl, theta, tag=f"mixed-scale N{N}")
    _check_eval(D, orc, wl, theta, split=1, tag=f"mixed-scale N{N}")

def test_cost_parity_ragged_batch(D, orc):
    wl = small_ragged(60, seed=7)
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=3)
    _check_eval(D, orc, wl, theta, tag="ragged")
    _check_eval(D, orc, wl, theta, split=8, tag="ragged")
    _check_eval(D, orc, wl, theta, split="tune", tag="ragged-autotuned")


def test_edge_cases_and_status(D, orc):
    wl = small_uniform(2, 64, 4, 8, seed=5)
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=1)
    theta[1, 2] = np.nan          # BADINPUT
    theta[2, 0] = 70.0            # |log10 tau| > 30: rejected
    theta[6, :] = 100.0           # rejected, and its group scale must not reach the valid lanes of its wave
    theta[3, 1] = theta[3, 0]     # duplicate tau: singular without damping
    theta[4, :] = [-11.0, -10.0, -9.0, -8.0]
    _check_eval(D, orc, wl, theta, damping=1e-8, tag="edge")
    wl2 = small_uniform(2, 64, 4, 8, seed=5)
    th2 = theta.copy()
    th2[[0, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15]] = [-11.5, -10.0, -8.5, -7.2]   # well conditioned
    _check_eval(D, orc, wl2, th2, damping=0.0, tag="edge-undamped")
    _check_eval(D, orc, wl, theta, damping=1e-8, flags=1, tag="edge-noflip")
    # a single frequency point, a single pole
    wl3 = small_uniform(3, 1, 1, 5, seed=2)
    th3 = W.draw_theta(wl3.cand_off, wl3.n_poles, wl3.lb, wl3.ub, 1, seed=2)
    _check_eval(D, orc, wl3, th3, tag="F1N1")


def test_empty_materials_and_determinism(D, orc):
    import torch
    wl = small_ragged(25, seed=11, Pr=(0, 3))
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=5)
    _check_eval(D, orc, wl, theta, tag="empty")
    wl = small_uniform(4, 500, 10, 64, seed=3)
    er, ei = targets_oracle(orc, wl)
    b = _gpu_batch(D, wl, er, ei)
    plan = D.Plan(b)
    th = torch.tensor(W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=2), device="cuda")
    c1 = D.fit_eval(plan, b, th)[0].clone()
    c2 = D.fit_eval(plan, b, th)[0].clone()
    assert torch.equal(c1, c2)
