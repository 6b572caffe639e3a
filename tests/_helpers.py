"""Shared helpers for the GPU parity tests: build the same seeded batch for the
oracle (CPU) and for the library (GPU), and the comparison rules."""
import numpy as np

import workloads as W

COST_RTOL = 1e-10      # cost relative error vs the FP64 oracle
WEIGHT_RTOL = 1e-8     # weights / eps_inf: max |diff| / max |ref| per candidate


def targets_oracle(orc, wl):
    return orc.material_eval(wl.kind, wl.params, wl.f_off, wl.omega, noise_seed=wl.noise_seed)


def cost_floor(wl, er, ei):
    """Scale below which a cost counts as zero: 1e-12 * sum(eps'^2 + eps''^2) of
    the candidate's material (exact-recovery cases have cost ~ 0)."""
    per_m = np.array([np.sum(er[wl.f_off[m]:wl.f_off[m + 1]] ** 2 + ei[wl.f_off[m]:wl.f_off[m + 1]] ** 2)
                      for m in range(wl.M)])
    P = np.diff(wl.cand_off)
    return 1e-12 * np.repeat(per_m, P)


def cost_rel_err(c, ref, floor):
    c = np.asarray(c)
    ref = np.asarray(ref)
    fin = np.isfinite(ref)
    out = np.zeros_like(ref)
    out[fin] = np.abs(c[fin] - ref[fin]) / np.maximum(np.abs(ref[fin]), floor[fin])
    # non-finite references must be reproduced exactly (inf stays inf, NaN stays NaN)
    bad = ~fin & ~((np.isnan(ref) & np.isnan(c)) | (ref == c))
    out[bad] = np.inf
    return out


def attributed_cost_err(orc, ob, theta, c_gpu, floor, damping, flags, rel64, stats=None):
    """Cost error after the oracle's judgement (oracle.judge_costs): a
    candidate over COST_RTOL against the FP64 oracle is judged against its
    80-bit instance, and its error is the one against that result.  Returns
    (errors, number of candidates judged against the 80-bit oracle)."""
    c64 = np.asarray(ob_cost64(orc, ob, theta, damping, flags))
    st = {}
    rel, _ = orc.judge_costs(ob, np.asarray(theta), c_gpu, c64, floor, COST_RTOL, damping, flags, st, rel=rel64)
    if stats is not None:
        stats.update(st)
    if st["over"]:
        print(f"over {COST_RTOL:g} against both oracles (index, err vs 80-bit, FP64 oracle vs 80-bit, cond*u): "
              f"{st['over']}", flush=True)
    return rel, st["oracle_limited"] + st["failed"]


def ob_cost64(orc, ob, theta, damping, flags):
    return orc.fit_eval(ob, theta, damping=damping, flags=flags)[0]


def weight_rel_err(w, ref, n_poles_per_cand):
    err = np.zeros(len(ref))
    for i, (a, r, n) in enumerate(zip(w, ref, n_poles_per_cand)):
        a, r = a[:n], r[:n]
        if not np.all(np.isfinite(r)):
            err[i] = 0.0 if np.array_equal(np.isnan(a), np.isnan(r)) else np.inf
            continue
        err[i] = np.max(np.abs(a - r)) / max(np.max(np.abs(r)), 1e-300)
    return err


def poles_per_cand(wl):
    return np.repeat(wl.n_poles, np.diff(wl.cand_off))


def small_uniform(M, F, N, P, seed, fmin=1e6, fmax=1e10, kinds=None):
    kind, params = W.draw_mixed(M, seed, fmin, fmax, kinds=kinds)
    lb, ub = W.tau_bounds(fmin, fmax)
    om = W.log_grid(fmin, fmax, F)
    return W.Workload(f"test M{M} F{F} N{N} P{P}", kind, params, W.offsets([F] * M), np.tile(om, M),
                      np.full(M, N, np.int32), W.offsets([P] * M), np.full(M, lb), np.full(M, ub), 1, seed=seed)


def mixed_scale_workload(N, F=150, P=37, seed=400, shift=-33):
    """Two materials with the same HN-family spectrum shape: one on the
    ordinary band, one on the band moved by `shift` decades (tau0 and the tau
    search box moved the other way).  With P not a multiple of the candidates
    per wave, tiles hold candidates of both."""
    import dataclasses
    a = small_uniform(1, F, N, P, seed=seed + N, kinds=[W.KIND_HN, W.KIND_CC, W.KIND_CD])
    params_b = a.params.copy()
    params_b[:, 2] *= 10.0 ** -shift
    return dataclasses.replace(
        a, name=f"{a.name} + band x1e{shift}", kind=np.concatenate([a.kind, a.kind]),
        params=np.concatenate([a.params, params_b]), f_off=W.offsets([F, F]),
        omega=np.concatenate([a.omega, a.omega * 10.0 ** shift]), n_poles=np.concatenate([a.n_poles, a.n_poles]),
        cand_off=W.offsets([P, P]), lb=np.concatenate([a.lb, a.lb - shift]), ub=np.concatenate([a.ub, a.ub - shift]))

def small_ragged(M, seed, Fr=(20, 700), Nr=(1, 24), Pr=(0, 150)):
    kind, params = W.draw_mixed(M, seed, 1e6, 1e10)
    g = W.rng(seed, 9)
    Fm = g.integers(Fr[0], Fr[1] + 1, size=M)
    Nm = g.integers(Nr[0], Nr[1] + 1, size=M).astype(np.int32)
    Pm = g.integers(Pr[0], Pr[1] + 1, size=M)
    lb, ub = W.tau_bounds(1e6, 1e10)
    om = np.concatenate([W.log_grid(1e6, 1e10, int(f)) for f in Fm])
    return W.Workload(f"ragged M{M}", kind, params, W.offsets(Fm), om, Nm, W.offsets(Pm), np.full(M, lb),
                      np.full(M, ub), 1, seed=seed)


def attributed_weight_err(orc, ob, theta, w_gpu, e_gpu, ok, npc, damping, flags, w64, e64):
    """Weight and eps_inf errors with the cost's judgement: a candidate over
    WEIGHT_RTOL against the FP64 oracle is judged against the 80-bit instance,
    and its errors are the ones against that result.  Returns (weight errors,
    eps_inf errors, n judged against the 80-bit oracle)."""
    werr = weight_rel_err(w_gpu[ok], w64[ok], npc[ok])
    eerr = np.abs(e_gpu[ok] - e64[ok]) / np.maximum(np.abs(e64[ok]), 1e-300)
    over = (werr > WEIGHT_RTOL) | (eerr > WEIGHT_RTOL)
    if not over.any():
        return werr, eerr, 0
    _, w80, e80, _ = orc.fit_eval(ob, theta, damping=damping, flags=flags, precision=80)
    werr[over] = weight_rel_err(w_gpu[ok][over], w80[ok][over], npc[ok][over])
    eerr[over] = (np.abs(e_gpu[ok] - e80[ok]) / np.maximum(np.abs(e80[ok]), 1e-300))[over]
    return werr, eerr, int(over.sum())
