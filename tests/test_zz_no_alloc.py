"""The allocation-free adjoint entry point (debye_fit_eval_grad_noalloc)
against debye_fit_eval_grad with a DEBYE_PLAN_TARGET_GRAD plan, through the
C ABI: two calls in a row, the second on a smaller batch, both bit-identical
to the ordinary entry point; a batch beyond the static workspace is refused
on the host."""
import numpy as np
import pytest

import workloads as W
from _helpers import small_ragged, targets_oracle

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.tensor(x, device="cuda")


def _case(D, orc, wl, seed):
    import torch
    er, ei = targets_oracle(orc, wl)
    b = D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, _t(er), _t(ei))
    th = _t(W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=seed))
    th = torch.nan_to_num(th, nan=-9.0)
    gc = _t(np.linspace(0.5, 2.0, wl.P))
    ref = D.fit_eval_grad(D.Plan(b, target_grads=True), b, th, grad_cost=gc, targets=True)
    torch.cuda.synchronize()
    plan = D.Plan(b)   # no target-gradient workspace in this plan
    got = D.fit_eval_grad(plan, b, th, grad_cost=gc, targets=True, noalloc=True)
    torch.cuda.synchronize()
    return ref, got


def test_noalloc_adjoint_equals_the_ordinary_entry_point(orc):
    import torch
    import paper_2109_01928_amd as D
    assert torch.cuda.is_available()
    big = small_ragged(24, seed=61, Fr=(50, 400), Nr=(2, 20), Pr=(10, 120))
    small = small_ragged(5, seed=62, Fr=(30, 120), Nr=(3, 9), Pr=(4, 30))
    assert small.P < big.P
    for wl, seed in ((big, 1), (small, 2)):
        print(f"[noalloc] {wl.name}: {wl.P} candidates, max N {wl.ld}", flush=True)
        ref, got = _case(D, orc, wl, seed)
        for name, a, b in zip(("cost", "grad_theta", "grad_re", "grad_im", "status"), ref, got):
            assert torch.equal(a, b), name
        assert torch.all(torch.isfinite(ref[1]))


def test_noalloc_rejects_batches_beyond_the_workspace(orc):
    import ctypes as C
    import torch
    import paper_2109_01928_amd as D
    # N = 20: 82 record doubles per candidate; 110,000 candidates need 72 MB > 64 MiB
    M, P, N, F = 2, 55_000, 20, 8
    om = W.log_grid(1e6, 1e10, F)
    z = np.zeros(M * F)
    b = D.Batch(W.offsets([F] * M), W.offsets([P] * M), np.full(M, N), np.tile(om, M), z, z)
    plan = D.Plan(b)
    th = torch.full((M * P, N), -9.0, dtype=torch.float64, device="cuda")
    with pytest.raises(D.DebyeError) as e:
        D.fit_eval_grad(plan, b, th, targets=True, noalloc=True)
    assert e.value.code == D.ERANGE and "static workspace" in str(e.value)
    # without target gradients nothing is needed from the workspace
    c, g, _, _, st = D.fit_eval_grad(plan, b, th, noalloc=True)
    torch.cuda.synchronize()
    assert torch.all(st == 0)
