"""DEBYE_FLAG_NO_REFINE: the weights from the damped Cholesky solve of the
normal equations alone, without the refinement step.

The oracle solves the damped least-squares problem of Sec. III-B by
Householder QR, so it is the accurate result the unrefined solve approximates.
The normal-equations solution differs from it by about cond(G^) u relative in
the weights, G^ being the column-scaled damped Gram matrix the kernel
factors.  The checks:
  - well-separated poles (cond(G^) computed here from the oracle's basis,
    at most 1e5): weights within 1e3 cond(G^) u of the oracle's (relative to
    the largest weight), costs within 1e-8, statuses equal;
  - random candidates (ill-conditioned ones included): statuses equal, costs
    finite wherever the oracle's are, and the damped least-squares objective
    of the unrefined signed weights is never below the oracle's minimum by
    more than rounding (the oracle's weights minimise it);
  - the adjoint accepts the flag and returns the same costs as the forward
    kernel with it;
  - unknown flag bits are refused."""
import numpy as np
import pytest

import workloads as W
from _helpers import cost_floor, cost_rel_err, small_ragged, small_uniform, targets_oracle

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
DAMP = 1e-8


@pytest.fixture(scope="module")
def D():
    import torch
    import paper_2109_01928_amd as D

    assert torch.cuda.is_available()
    D.lib()
    return D


def _run(D, wl, er, ei, theta, flags):
    import torch
    b = D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, torch.tensor(er, device="cuda"),
                torch.tensor(ei, device="cuda"))
    plan = D.Plan(b)
    out = D.fit_eval(plan, b, torch.tensor(theta, device="cuda"), damping=DAMP, flags=flags)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def _scaled_gram_cond(orc, omega, th):
    _, I = orc.basis(omega, th)
    G = I @ I.T
    d = np.sqrt(np.diag(G))
    Gs = G / np.outer(d, d) + DAMP * np.eye(len(th))
    return np.linalg.cond(Gs)


def _objective(orc, omega, ei, th, z):
    """||I z - eps''||^2 + damping sum (||I_i|| z_i)^2, the problem the
    weights solve (Marquardt scaling)."""
    _, I = orc.basis(omega, th)
    r = I.T @ z - ei
    return float(r @ r + DAMP * np.sum((np.linalg.norm(I, axis=1) * z) ** 2))


def test_no_refine_matches_oracle_on_well_separated_poles(D, orc):
    wl = small_uniform(6, 400, 8, 40, seed=71)
    er, ei = targets_oracle(orc, wl)
    g = W.rng(71, 3)
    base = np.linspace(wl.lb[0] + 0.5, wl.ub[0] - 0.5, 8)   # 0.57 decades apart
    theta = base[None, :] + g.uniform(-0.05, 0.05, size=(wl.P, 8))
    ob = orc.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, er, ei)
    oc, ow, oe, ost = orc.fit_eval(ob, theta, damping=DAMP)
    c, w, e, st = _run(D, wl, er, ei, theta, D.FLAG_NO_REFINE)
    np.testing.assert_array_equal(st, ost)
    om = wl.omega[:400]
    worst = 0.0
    for i in range(wl.P):
        kappa = _scaled_gram_cond(orc, om, theta[i])
        assert kappa <= 1e5, kappa
        scale = np.max(np.abs(ow[i, :8]))
        err = np.max(np.abs(w[i, :8] - ow[i, :8])) / scale
        assert err <= 1e3 * kappa * U, (i, err, kappa)
        worst = max(worst, err / (kappa * U))
    rel = cost_rel_err(c, oc, cost_floor(wl, er, ei))
    print(f"[no-refine, separated] max weight error / (cond u) {worst:.2f}, max cost rel err {rel.max():.2e}")
    assert rel.max() <= 1e-8


def test_no_refine_random_candidates(D, orc):
    wl = small_ragged(10, seed=72, Fr=(40, 400), Nr=(1, 20), Pr=(5, 60))
    er, ei = targets_oracle(orc, wl)
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=72)
    ob = orc.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, er, ei)
    flags = D.FLAG_NO_REFINE | D.FLAG_NO_SIGN_FLIP   # signed weights: the least-squares solution itself
    oc, oz, _, ost = orc.fit_eval(ob, theta, damping=DAMP, flags=flags)
    c, z, _, st = _run(D, wl, er, ei, theta, flags)
    np.testing.assert_array_equal(st, ost)
    assert np.all(np.isfinite(c[np.isfinite(oc)]))
    below = 0.0
    for m in range(wl.M):
        f0, f1 = wl.f_off[m], wl.f_off[m + 1]
        n = wl.n_poles[m]
        scale = float(ei[f0:f1] @ ei[f0:f1])
        for i in range(wl.cand_off[m], wl.cand_off[m + 1]):
            if ost[i] != 0:
                continue
            phi_gpu = _objective(orc, wl.omega[f0:f1], ei[f0:f1], theta[i, :n], z[i, :n])
            phi_orc = _objective(orc, wl.omega[f0:f1], ei[f0:f1], theta[i, :n], oz[i, :n])
            below = max(below, (phi_orc - phi_gpu) / scale)
    print(f"[no-refine, random] largest drop of the objective below the oracle's minimum: {below:.2e} of ||eps''||^2")
    assert below <= 1e-12


def test_no_refine_adjoint_and_flag_check(D, orc):
    import torch
    wl = small_uniform(3, 200, 12, 30, seed=73)
    er, ei = targets_oracle(orc, wl)
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=73)
    b = D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, torch.tensor(er, device="cuda"),
                torch.tensor(ei, device="cuda"))
    plan = D.Plan(b)
    th = torch.tensor(theta, device="cuda")
    c_fwd = D.fit_eval(plan, b, th, damping=DAMP, flags=D.FLAG_NO_REFINE, want_weights=False)[0]
    c_adj = D.fit_eval_grad(plan, b, th, damping=DAMP, flags=D.FLAG_NO_REFINE)[0]
    c_ref = D.fit_eval(plan, b, th, damping=DAMP, want_weights=False)[0]
    torch.cuda.synchronize()
    rel = cost_rel_err(c_adj.cpu().numpy(), c_fwd.cpu().numpy(), cost_floor(wl, er, ei))
    assert rel.max() <= 1e-10, rel.max()
    assert not torch.equal(c_fwd, c_ref)   # the refinement changes the result
    with pytest.raises(D.DebyeError):
        D.fit_eval(plan, b, th, damping=DAMP, flags=8)
