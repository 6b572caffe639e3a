"""CPU oracle for the multi-pole Debye fitting method (test infrastructure).

This package is the plain FP64 reference that the GPU library is checked
against.  Only the test suite, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import it; the GPU library never does, and
the two share no code.  The arithmetic lives in ``debye_oracle.cpp`` (built to
``liboracle.so`` by ``oracle/build.py``); this module only marshals numpy
arrays through ctypes.

Paper: Majchrowska et al., "Modelling Arbitrary Complex Dielectric Properties
- an automated implementation for gprMax", Sec. II-B (Eqs. 1, 3-7) and
Sec. III (fitting procedure).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ST_OK, ST_BADINPUT, ST_SINGULAR = 0, 1, 2
FLAG_NO_SIGN_FLIP = 1
KIND_DEBYE, KIND_HN, KIND_CC, KIND_CD, KIND_JONSCHER, KIND_CRIM, KIND_HNSUM = range(7)
PARAM_STRIDE = 16

_d = C.POINTER(C.c_double)
_i64 = C.POINTER(C.c_int64)
_i32 = C.POINTER(C.c_int32)
_i8 = C.POINTER(C.c_int8)
_u64 = C.POINTER(C.c_uint64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.orc_philox4x64_10.argtypes = [_u64, _u64, _u64]
        L.orc_material_eval.argtypes = [C.c_int32, _i8, _d, _i64, _d, C.c_uint64, _d, _d, _d, C.c_int]
        L.orc_basis.argtypes = [_d, C.c_int64, _d, C.c_int32, _d, _d]
        L.orc_fit_eval_batch.argtypes = [C.c_int32, _i64, _i64, _i32, _d, _d, _d, _d, C.c_int64,
                                         C.c_double, C.c_uint32, _d, _d, _d, _i8, C.c_int32, C.c_int]
        L.orc_fit_grad_batch.argtypes = [C.c_int32, _i64, _i64, _i32, _d, _d, _d, _d, C.c_int64,
                                         C.c_double, C.c_uint32, _d, _d, _d, _d, _d, _i8, C.c_int]
        L.orc_fit_cs_grad.argtypes = [C.c_int64, _d, _d, _d, C.c_int32, _d, C.c_double, C.c_uint32,
                                      C.c_double, _d, _d, _d]
        L.orc_fit_detail.argtypes = [C.c_int64, _d, _d, _d, C.c_int32, _d, C.c_double, C.c_uint32,
                                     _d, _d, _d, _d]
        L.orc_pso_init.argtypes = [C.c_int32, _i64, _i32, C.c_int64, _d, _d, C.c_uint64,
                                   _d, _d, _d, _d, _d, _i64]
        L.orc_pso_step.argtypes = [C.c_int32, _i64, _i32, C.c_int64, _d, _d, C.c_double, C.c_double,
                                   C.c_double, C.c_uint64, C.c_int32, C.c_int32, _d, _d, _d, _d, _d,
                                   _d, _d, _i64, _d, C.c_int64]
        L.orc_lbfgs_batch.argtypes = [C.c_int32, _i64, _i32, _d, _d, _d, _d, C.c_int64, _d, _d, C.c_double,
                                      C.c_uint32, C.c_int32, C.c_int32, C.c_int32, C.c_double, _d, _i32, C.c_int]
        L.orc_lbfgs_two_loop.argtypes = [C.c_int32, C.c_int32, _d, _d, _d, _d]
        L.orc_afe.argtypes = [C.c_int64, _d, _d, _d, C.c_int32, _d, _d, C.c_double]
        L.orc_afe.restype = C.c_double
        L.orc_fit_from_basis.argtypes = [C.c_int64, _d, _d, _d, _d, C.c_int32, C.c_double, C.c_uint32, C.c_int32,
                                         _d]
        L.orc_fit_cond.argtypes = [C.c_int64, _d, _d, _d, C.c_int32, _d, C.c_double, C.c_uint32, _d, _d, _d]
        L.orc_de_init.argtypes = [C.c_int32, _i64, _i32, C.c_int64, _d, _d, C.c_uint64, _d, _d, _d, _i64]
        L.orc_de_trial.argtypes = [C.c_int32, _i64, _i32, C.c_int64, _d, _d, C.c_double, C.c_double, C.c_double,
                                   C.c_uint64, C.c_int32, _d, _d]
        L.orc_de_select.argtypes = [C.c_int32, _i64, _i32, C.c_int64, C.c_int32, _d, _d, _d, _d, _d, _d, _i64, _d,
                                    C.c_int64]
        L.orc_series_exp_log.argtypes = [C.c_int64, _d, _d, _d]
        L.orc_student_t.argtypes = [C.c_uint64, C.c_int64, C.c_double, _d]
        L.orc_da_temps.argtypes = [C.c_double, C.c_double, C.c_int32, _d, _d]
        L.orc_da_init.argtypes = [C.c_int32, _i64, _i32, C.c_int64, _d, _d, C.c_uint64, _d, _d, _d, _i64]
        L.orc_da_visit.argtypes = [C.c_int32, _i64, _i32, C.c_int64, _d, _d, C.c_double, C.c_double, C.c_uint64,
                                   C.c_int32, _d, _d]
        L.orc_da_accept.argtypes = [C.c_int32, _i64, _i32, C.c_int64, C.c_double, C.c_double, C.c_double,
                                    C.c_uint64, C.c_int32, _d, _d, _d, _d, _d, _d, _i64, _d, C.c_int64]
        L.orc_material_eval_idx.argtypes = [C.c_int32, _i8, _d, _i64, _d, C.c_uint64, _i64, _d, _d, C.c_int]
        L.orc_fit_cond_batch.argtypes = [C.c_int32, _i64, _i64, _i32, _d, _d, _d, _d, C.c_int64, C.c_double,
                                         C.c_uint32, _d, C.c_int]
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a, t):
    if a is None:
        return None
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return lib().orc_num_threads()


# ---------------------------------------------------------------------------
def philox4x64_10(ctr, key):
    """Philox4x64-10 block for counter ctr[4] and key key[2] (uint64)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_p(c, _u64), _p(k, _u64), _p(out, _u64))
    return out


def material_eval(kind, params, f_off, omega, noise_seed=0, jac=False, nthreads=0):
    """Targets eps', eps'' (and optionally d(eps',eps'')/d(eps_inf,d_eps,tau0,alpha,beta)
    as [F_tot][5][2]) for a ragged batch of materials (Eqs. 3-6)."""
    kind = np.ascontiguousarray(kind, dtype=np.int8)
    params = _f64(params).reshape(-1, PARAM_STRIDE)
    f_off = np.ascontiguousarray(f_off, dtype=np.int64)
    omega = _f64(omega)
    M = len(kind)
    Ft = int(f_off[-1])
    er = np.empty(Ft)
    ei = np.empty(Ft)
    J = np.empty((Ft, 5, 2)) if jac else None
    rc = lib().orc_material_eval(M, _p(kind, _i8), _p(params, _d), _p(f_off, _i64), _p(omega, _d),
                                 C.c_uint64(noise_seed), _p(er, _d), _p(ei, _d), _p(J, _d), nthreads)
    if rc != 0:
        raise ValueError("material_eval: unknown material kind")
    return (er, ei, J) if jac else (er, ei)


def material_eval_sample(kind, params, f_off, omega, mat_index, noise_seed=0, nthreads=0):
    """Targets of a sample of a batch's materials: material m of the arguments
    draws its noise as material mat_index[m] of the full batch."""
    kind = np.ascontiguousarray(kind, dtype=np.int8)
    params = _f64(params).reshape(-1, PARAM_STRIDE)
    f_off = np.ascontiguousarray(f_off, dtype=np.int64)
    idx = np.ascontiguousarray(mat_index, dtype=np.int64)
    omega = _f64(omega)
    er = np.empty(int(f_off[-1]))
    ei = np.empty(int(f_off[-1]))
    rc = lib().orc_material_eval_idx(len(kind), _p(kind, _i8), _p(params, _d), _p(f_off, _i64), _p(omega, _d),
                                     C.c_uint64(noise_seed), _p(idx, _i64), _p(er, _d), _p(ei, _d), nthreads)
    if rc != 0:
        raise ValueError("material_eval: unknown material kind")
    return er, ei


def basis(omega, theta):
    """Re/Im Debye basis [N][F] for one candidate (Eq. 7 with Eq. 1's sign)."""
    omega = _f64(omega)
    theta = _f64(theta)
    N, F = len(theta), len(omega)
    re_ = np.empty((N, F))
    im_ = np.empty((N, F))
    lib().orc_basis(_p(omega, _d), F, _p(theta, _d), N, _p(re_, _d), _p(im_, _d))
    return re_, im_


class Batch:
    """Host description of a ragged batch: material m owns frequencies
    f_off[m]:f_off[m+1] and candidates cand_off[m]:cand_off[m+1]; candidate c
    stores its log10 tau in theta[c, :n_poles[m]] (row stride ld)."""

    def __init__(self, f_off, cand_off, n_poles, omega, eps_re, eps_im):
        self.f_off = np.ascontiguousarray(f_off, dtype=np.int64)
        self.cand_off = np.ascontiguousarray(cand_off, dtype=np.int64)
        self.n_poles = np.ascontiguousarray(n_poles, dtype=np.int32)
        self.omega = _f64(omega)
        self.eps_re = _f64(eps_re)
        self.eps_im = _f64(eps_im)
        self.M = len(self.n_poles)
        self.P = int(self.cand_off[-1])


def fit_eval(b: Batch, theta, damping=1e-8, flags=0, precision=64, nthreads=0):
    """Cost, flipped weights (Delta eps), eps_inf and status for every candidate."""
    theta = _f64(theta)
    ld = theta.shape[1]
    P = b.P
    cost = np.empty(P)
    eps_inf = np.empty(P)
    w = np.full((P, ld), np.nan)
    st = np.empty(P, dtype=np.int8)
    lib().orc_fit_eval_batch(b.M, _p(b.f_off, _i64), _p(b.cand_off, _i64), _p(b.n_poles, _i32),
                             _p(b.omega, _d), _p(b.eps_re, _d), _p(b.eps_im, _d), _p(theta, _d), ld,
                             damping, flags, _p(cost, _d), _p(w, _d), _p(eps_inf, _d), _p(st, _i8),
                             precision, nthreads)
    return cost, w, eps_inf, st


def fit_grad(b: Batch, theta, damping=1e-8, flags=0, grad_cost=None, nthreads=0):
    """Cost and the adjoint gradient: d cost/d log10 tau [P][ld] and the target
    gradients summed over each material's candidates (weighted by grad_cost)."""
    theta = _f64(theta)
    ld = theta.shape[1]
    P = b.P
    cost = np.empty(P)
    gt = np.full((P, ld), np.nan)
    gr = np.empty(len(b.omega))
    gi = np.empty(len(b.omega))
    st = np.empty(P, dtype=np.int8)
    gc = None if grad_cost is None else _f64(grad_cost)
    lib().orc_fit_grad_batch(b.M, _p(b.f_off, _i64), _p(b.cand_off, _i64), _p(b.n_poles, _i32),
                             _p(b.omega, _d), _p(b.eps_re, _d), _p(b.eps_im, _d), _p(theta, _d), ld,
                             damping, flags, _p(gc, _d), _p(cost, _d), _p(gt, _d), _p(gr, _d),
                             _p(gi, _d), _p(st, _i8), nthreads)
    return cost, gt, gr, gi, st


def fit_cs_grad(omega, eps_re, eps_im, theta, damping=1e-8, flags=0, h=1e-30, targets=True):
    """Complex-step derivatives of one candidate's cost."""
    omega, eps_re, eps_im, theta = map(_f64, (omega, eps_re, eps_im, theta))
    F, N = len(omega), len(theta)
    gt = np.empty(N)
    gr = np.empty(F) if targets else None
    gi = np.empty(F) if targets else None
    lib().orc_fit_cs_grad(F, _p(omega, _d), _p(eps_re, _d), _p(eps_im, _d), N, _p(theta, _d),
                          damping, flags, h, _p(gt, _d), _p(gr, _d), _p(gi, _d))
    return (gt, gr, gi) if targets else gt


def fit_detail(omega, eps_re, eps_im, theta, damping=1e-8, flags=0):
    """Unflipped LS solution z, scaling d and residuals of one candidate."""
    omega, eps_re, eps_im, theta = map(_f64, (omega, eps_re, eps_im, theta))
    F, N = len(omega), len(theta)
    z, d, rr, ri = np.empty(N), np.empty(N), np.empty(F), np.empty(F)
    st = lib().orc_fit_detail(F, _p(omega, _d), _p(eps_re, _d), _p(eps_im, _d), N, _p(theta, _d),
                              damping, flags, _p(z, _d), _p(d, _d), _p(rr, _d), _p(ri, _d))
    return st, z, d, rr, ri


def fit_from_basis(R, I, eps_re, eps_im, damping=1e-8, flags=0, precision=64):
    """Cost of one candidate from an explicitly given basis R, I [F][N]
    (steps 2-5 of the forward map)."""
    R, I, eps_re, eps_im = map(_f64, (R, I, eps_re, eps_im))
    F, N = R.shape
    cost = np.empty(1)
    st = lib().orc_fit_from_basis(F, _p(R, _d), _p(I, _d), _p(eps_re, _d), _p(eps_im, _d), N, damping, flags,
                                  precision, _p(cost, _d))
    return cost[0], st


def fit_cond(omega, eps_re, eps_im, theta, damping=1e-8, flags=0):
    """Relative condition number of one candidate's cost under componentwise
    relative perturbations of the basis, and the total derivatives dC/dR,
    dC/dI [F][N] it is built from (80-bit arithmetic)."""
    omega, eps_re, eps_im, theta = map(_f64, (omega, eps_re, eps_im, theta))
    F, N = len(omega), len(theta)
    dR, dI, cond = np.empty((F, N)), np.empty((F, N)), np.empty(1)
    st = lib().orc_fit_cond(F, _p(omega, _d), _p(eps_re, _d), _p(eps_im, _d), N, _p(theta, _d), damping, flags,
                            _p(dR, _d), _p(dI, _d), _p(cond, _d))
    return cond[0], dR, dI, st


def fit_cond_batch(b: Batch, theta, damping=1e-8, flags=0, nthreads=0):
    """fit_cond's condition number for every candidate of a batch."""
    theta = _f64(theta)
    cond = np.empty(b.P)
    lib().orc_fit_cond_batch(b.M, _p(b.f_off, _i64), _p(b.cand_off, _i64), _p(b.n_poles, _i32),
                             _p(b.omega, _d), _p(b.eps_re, _d), _p(b.eps_im, _d), _p(theta, _d),
                             theta.shape[1], damping, flags, _p(cond, _d), nthreads)
    return cond


UNIT_ROUNDOFF = 2.0 ** -53


def judge_costs(b: Batch, theta, c_test, c64, floor, rtol, damping=1e-8, flags=0, stats=None, rel=None):
    """Parity judgement of costs computed elsewhere against this oracle.

    The error of a candidate is its relative error (floored) against the FP64
    oracle.  A candidate above rtol there is re-judged against the 80-bit
    instance of the oracle (the more accurate reference; the FP64 oracle's own
    error can exceed rtol on ill-conditioned candidates): its error is then
    the one against the 80-bit result, and it counts as "oracle_limited" if
    that is within rtol.  No other allowance: a candidate passes only if it
    is within rtol of the FP64 or of the 80-bit oracle.  For each candidate
    still above rtol, stats["over"] lists (index, error vs 80-bit, error of
    the FP64 oracle vs 80-bit, cond * u) as a diagnosis (cond from fit_cond:
    the cost's sensitivity to rounding the basis).  `rel` (optional) holds
    precomputed errors against the FP64 oracle; only candidates with a finite
    FP64 cost are re-judged.  Returns (errors, stats)."""
    c_test, c64, floor = map(np.asarray, (c_test, c64, floor))
    if rel is None:
        rel = np.abs(c_test - c64) / np.maximum(c64, floor)
    rel = np.array(rel, dtype=np.float64)
    st = dict(n=len(rel), oracle_limited=0, failed=0, max_rel_80=0.0, over=[])
    over = np.nonzero(~(rel <= rtol) & np.isfinite(c64))[0]
    if len(over):
        idx = np.searchsorted(b.cand_off, over, side="right") - 1
        for c, m in zip(over, idx):
            f0, f1 = b.f_off[m], b.f_off[m + 1]
            one = Batch([0, f1 - f0], [0, 1], b.n_poles[m:m + 1], b.omega[f0:f1], b.eps_re[f0:f1],
                        b.eps_im[f0:f1])
            th = theta[c:c + 1]
            c80 = fit_eval(one, th, damping, flags, precision=80)[0][0]
            r80 = abs(c_test[c] - c80) / max(c80, floor[c])
            st["max_rel_80"] = max(st["max_rel_80"], float(r80))
            rel[c] = r80
            if r80 <= rtol:
                st["oracle_limited"] += 1
                continue
            st["failed"] += 1
            own = abs(c64[c] - c80) / max(c80, floor[c])
            cond = fit_cond(b.omega[f0:f1], b.eps_re[f0:f1], b.eps_im[f0:f1], th[0, :b.n_poles[m]], damping,
                            flags)[0]
            st["over"].append((int(c), float(r80), float(own), float(cond * UNIT_ROUNDOFF)))
    if stats is not None:
        stats.update(st)
    return rel, st


class Swarm:
    """PSO state in the library's layout (rows of stride ld)."""

    def __init__(self, P, M, ld, hist_len=0):
        self.x = np.zeros((P, ld))
        self.v = np.zeros((P, ld))
        self.pbest_x = np.zeros((P, ld))
        self.pbest_cost = np.zeros(P)
        self.gbest_x = np.zeros((M, ld))
        self.gbest_cost = np.zeros(M)
        self.gbest_idx = np.zeros(M, dtype=np.int64)
        self.history = np.full((M, max(hist_len, 1)), np.nan)

    def copy(self):
        s = Swarm.__new__(Swarm)
        for k, v in self.__dict__.items():
            setattr(s, k, v.copy())
        return s


def pso_init(cand_off, n_poles, lb, ub, seed, sw: Swarm):
    cand_off = np.ascontiguousarray(cand_off, dtype=np.int64)
    n_poles = np.ascontiguousarray(n_poles, dtype=np.int32)
    lb, ub = _f64(lb), _f64(ub)
    lib().orc_pso_init(len(n_poles), _p(cand_off, _i64), _p(n_poles, _i32), sw.x.shape[1], _p(lb, _d),
                       _p(ub, _d), C.c_uint64(seed), _p(sw.x, _d), _p(sw.v, _d), _p(sw.pbest_x, _d),
                       _p(sw.pbest_cost, _d), _p(sw.gbest_cost, _d), _p(sw.gbest_idx, _i64))


def pso_step(cand_off, n_poles, lb, ub, inertia, c1, c2, seed, t, move, cost, sw: Swarm):
    cand_off = np.ascontiguousarray(cand_off, dtype=np.int64)
    n_poles = np.ascontiguousarray(n_poles, dtype=np.int32)
    lb, ub, cost = _f64(lb), _f64(ub), _f64(cost)
    lib().orc_pso_step(len(n_poles), _p(cand_off, _i64), _p(n_poles, _i32), sw.x.shape[1], _p(lb, _d),
                       _p(ub, _d), inertia, c1, c2, C.c_uint64(seed), t, int(move), _p(cost, _d),
                       _p(sw.x, _d), _p(sw.v, _d), _p(sw.pbest_x, _d), _p(sw.pbest_cost, _d),
                       _p(sw.gbest_x, _d), _p(sw.gbest_cost, _d), _p(sw.gbest_idx, _i64),
                       _p(sw.history, _d), sw.history.shape[1])


def pso_run(b: Batch, lb, ub, iters, inertia=0.7, c1=1.5, c2=1.5, seed=0, ld=None, damping=1e-8,
            flags=0, nthreads=0):
    """Whole swarm fit: init, evaluate, then `iters` x (move + evaluate), then a
    final bests-only step.  P*(iters+1) evaluations per material."""
    ld = ld or int(b.n_poles.max())
    sw = Swarm(b.P, b.M, ld, iters + 1)
    pso_init(b.cand_off, b.n_poles, lb, ub, seed, sw)
    cost = fit_eval(b, sw.x, damping, flags, nthreads=nthreads)[0]
    for t in range(1, iters + 1):
        pso_step(b.cand_off, b.n_poles, lb, ub, inertia, c1, c2, seed, t, True, cost, sw)
        cost = fit_eval(b, sw.x, damping, flags, nthreads=nthreads)[0]
    pso_step(b.cand_off, b.n_poles, lb, ub, inertia, c1, c2, seed, iters + 1, False, cost, sw)
    return sw


class Population:
    """Differential-evolution state in the library's layout (rows of stride ld)."""

    def __init__(self, P, M, ld, hist_len=0):
        self.x = np.zeros((P, ld))
        self.u = np.zeros((P, ld))
        self.fit = np.zeros(P)
        self.best_x = np.zeros((M, ld))
        self.best_cost = np.zeros(M)
        self.best_idx = np.zeros(M, dtype=np.int64)
        self.history = np.full((M, max(hist_len, 1)), np.nan)


def de_init(cand_off, n_poles, lb, ub, seed, pop: Population):
    cand_off = np.ascontiguousarray(cand_off, np.int64)
    n_poles = np.ascontiguousarray(n_poles, np.int32)
    lib().orc_de_init(len(n_poles), _p(cand_off, _i64), _p(n_poles, _i32), pop.x.shape[1], _p(_f64(lb), _d),
                      _p(_f64(ub), _d), seed, _p(pop.x, _d), _p(pop.fit, _d), _p(pop.best_cost, _d),
                      _p(pop.best_idx, _i64))


def de_trial(cand_off, n_poles, lb, ub, f_lo, f_hi, cr, seed, t, pop: Population):
    """Trial vectors of generation t into pop.u (DE/rand/1/bin); a population
    of fewer than 4 members gets its targets as trials."""
    cand_off = np.ascontiguousarray(cand_off, np.int64)
    n_poles = np.ascontiguousarray(n_poles, np.int32)
    lib().orc_de_trial(len(n_poles), _p(cand_off, _i64), _p(n_poles, _i32), pop.x.shape[1], _p(_f64(lb), _d),
                       _p(_f64(ub), _d), f_lo, f_hi, cr, seed, t, _p(pop.x, _d), _p(pop.u, _d))


def de_select(cand_off, n_poles, t, u, cost_u, pop: Population):
    cand_off = np.ascontiguousarray(cand_off, np.int64)
    n_poles = np.ascontiguousarray(n_poles, np.int32)
    u = _f64(u)
    cost_u = _f64(cost_u)
    lib().orc_de_select(len(n_poles), _p(cand_off, _i64), _p(n_poles, _i32), pop.x.shape[1], t, _p(u, _d),
                        _p(cost_u, _d), _p(pop.x, _d), _p(pop.fit, _d), _p(pop.best_x, _d), _p(pop.best_cost, _d),
                        _p(pop.best_idx, _i64), _p(pop.history, _d), pop.history.shape[1])


def de_run(b: Batch, lb, ub, iters, f_lo=0.5, f_hi=1.0, cr=0.7, seed=0, ld=None, damping=1e-8, flags=0,
           nthreads=0):
    """Whole DE fit: init, evaluate the initial population (generation 0),
    then `iters` x (trials, evaluate, select).  P*(iters+1) evaluations."""
    ld = ld or int(b.n_poles.max())
    pop = Population(b.P, b.M, ld, iters + 1)
    de_init(b.cand_off, b.n_poles, lb, ub, seed, pop)
    de_select(b.cand_off, b.n_poles, 0, pop.x.copy(), fit_eval(b, pop.x, damping, flags, nthreads=nthreads)[0], pop)
    for t in range(1, iters + 1):
        de_trial(b.cand_off, b.n_poles, lb, ub, f_lo, f_hi, cr, seed, t, pop)
        de_select(b.cand_off, b.n_poles, t, pop.u, fit_eval(b, pop.u, damping, flags, nthreads=nthreads)[0], pop)
    return pop


def lbfgs(b: Batch, theta, lb, ub, steps=50, mem=10, max_trials=30, c1=1e-4, damping=1e-8, flags=0,
          nthreads=0, rejected=False):
    """L-BFGS polish of one candidate per material (theta[M][ld]) inside the
    box [lb[m], ub[m]]; returns the polished theta and the cost history
    [M][steps+1] (and, with rejected=True, the number of accepted steps per
    material whose curvature pair s.y <= 1e-300 was not stored while the
    history held `mem` pairs)."""
    th = _f64(theta).copy()
    lb = _f64(np.broadcast_to(lb, (b.M,)))
    ub = _f64(np.broadcast_to(ub, (b.M,)))
    hist = np.empty((b.M, steps + 1))
    rej = np.zeros(b.M, dtype=np.int32)
    lib().orc_lbfgs_batch(b.M, _p(b.f_off, _i64), _p(b.n_poles, _i32), _p(b.omega, _d), _p(b.eps_re, _d),
                          _p(b.eps_im, _d), _p(th, _d), th.shape[1], _p(lb, _d), _p(ub, _d), damping, flags,
                          steps, mem, max_trials, c1, _p(hist, _d), _p(rej, _i32), nthreads)
    return (th, hist, rej) if rejected else (th, hist)


def lbfgs_two_loop(S, Y, v):
    """H v of the L-BFGS two-loop recursion (the polish's search direction is
    -H g) for the pairs S, Y [n][N] (oldest first)."""
    S, Y, v = map(_f64, (S, Y, v))
    n, N = S.shape if S.ndim == 2 else (0, len(v))
    out = np.empty(N)
    lib().orc_lbfgs_two_loop(N, n, _p(S.reshape(-1) if n else np.zeros(1), _d), _p(Y.reshape(-1) if n else np.zeros(1), _d),
                             _p(v, _d), _p(out, _d))
    return out


def afe(omega, eps_re, eps_im, d_eps, tau, eps_inf):
    """Average fractional error (percent) of a fitted multi-Debye model (Sec. IV)."""
    omega, eps_re, eps_im, d_eps, tau = map(_f64, (omega, eps_re, eps_im, d_eps, tau))
    return lib().orc_afe(len(omega), _p(omega, _d), _p(eps_re, _d), _p(eps_im, _d), len(d_eps),
                         _p(d_eps, _d), _p(tau, _d), float(eps_inf))


def fit_auto(f_off, omega, eps_re, eps_im, lb, ub, n_min=1, n_max=20, afe_target=5.0, particles=64, iters=100,
             inertia=0.7, c1=1.5, c2=1.5, seed=0, polish_steps=20, damping=1e-8, flags=0, nthreads=0):
    """Automatic pole count (Sec. III-B), one pole count at a time as the paper
    describes it: N = n_min, n_min + 1, ... until the average fractional error
    of the fit is below afe_target (percent), or N = n_max.  The fit of
    material m with N poles is a swarm of `particles` for `iters` iterations
    with Philox key (seed, m * NN + N - n_min), NN = n_max - n_min + 1 (the
    swarm of a batch entry at that index; the other entries of the batch are
    empty), then `polish_steps` L-BFGS steps (memory 10, 30 trials, c1 = 1e-4)
    on its best.  Returns (N [M], log10_tau [M][n_max], weights [M][n_max],
    eps_inf [M], afe [M])."""
    f_off = np.ascontiguousarray(f_off, np.int64)
    omega, eps_re, eps_im = map(_f64, (omega, eps_re, eps_im))
    M = len(f_off) - 1
    lb = _f64(np.broadcast_to(lb, (M,)))
    ub = _f64(np.broadcast_to(ub, (M,)))
    NN = n_max - n_min + 1
    E = M * NN
    out_n = np.zeros(M, np.int32)
    out_th = np.full((M, n_max), np.nan)
    out_w = np.full((M, n_max), np.nan)
    out_e = np.full(M, np.nan)
    out_a = np.full(M, np.nan)
    todo = list(range(M))
    for N in range(n_min, n_max + 1):
        if not todo:
            break
        # the full entry batch: only (m, N) of unresolved m carry particles
        active = np.zeros(E, bool)
        for m in todo:
            active[m * NN + (N - n_min)] = True
        ent_m = np.arange(E) // NN
        F_e = np.where(active, np.diff(f_off)[ent_m], 1)
        P_e = np.where(active, particles, 0)
        fe = np.concatenate([[0], np.cumsum(F_e)])
        src = np.concatenate([np.arange(f_off[m], f_off[m] + F_e[e]) for e, m in enumerate(ent_m)])
        b = Batch(fe, np.concatenate([[0], np.cumsum(P_e)]), np.full(E, N, np.int32), omega[src], eps_re[src],
                  eps_im[src])
        sw = pso_run(b, lb[ent_m], ub[ent_m], iters, inertia, c1, c2, seed, ld=N, damping=damping, flags=flags,
                     nthreads=nthreads)
        for m in list(todo):
            e = m * NN + (N - n_min)
            a, z = f_off[m], f_off[m + 1]
            one = Batch([0, z - a], [0, 1], [N], omega[a:z], eps_re[a:z], eps_im[a:z])
            th = sw.gbest_x[e:e + 1, :N].copy()
            if polish_steps > 0:
                th, _ = lbfgs(one, th, lb[m], ub[m], steps=polish_steps, mem=10, max_trials=30, c1=1e-4,
                              damping=damping, flags=flags)
            c, w, einf, st = fit_eval(one, th, damping, flags)
            err = afe(omega[a:z], eps_re[a:z], eps_im[a:z], w[0, :N], 10.0 ** th[0], einf[0])
            if err < afe_target or N == n_max:
                out_n[m] = N
                out_th[m, :N] = th[0]
                out_w[m, :N] = w[0, :N]
                out_e[m] = einf[0]
                out_a[m] = err
                todo.remove(m)
    return out_n, out_th, out_w, out_e, out_a


# ---------------------------------------------------------------------------
# Annealing (generalized simulated annealing, batched Markov chains)
# ---------------------------------------------------------------------------
DA_QV, DA_QA, DA_T0 = 2.62, -5.0, 5230.0


def series_exp_log(x):
    """The oracle's own exp and log (series with every operation rounded)."""
    x = _f64(np.atleast_1d(x))
    ex, lg = np.empty_like(x), np.empty_like(x)
    lib().orc_series_exp_log(len(x), _p(x, _d), _p(ex, _d), _p(lg, _d))
    return ex, lg


def student_t(seed, n, nu):
    """n draws of the annealing's visiting variate (Student-t, nu degrees of freedom)."""
    out = np.empty(n)
    lib().orc_student_t(seed, n, nu, _p(out, _d))
    return out


def da_temps(t, qv=DA_QV, t0=DA_T0):
    vs, ta = C.c_double(), C.c_double()
    lib().orc_da_temps(qv, t0, t, C.byref(vs), C.byref(ta))
    return vs.value, ta.value


def da_init(cand_off, n_poles, lb, ub, seed, pop: Population):
    cand_off = np.ascontiguousarray(cand_off, np.int64)
    n_poles = np.ascontiguousarray(n_poles, np.int32)
    lib().orc_da_init(len(n_poles), _p(cand_off, _i64), _p(n_poles, _i32), pop.x.shape[1], _p(_f64(lb), _d),
                      _p(_f64(ub), _d), seed, _p(pop.x, _d), _p(pop.fit, _d), _p(pop.best_cost, _d),
                      _p(pop.best_idx, _i64))


def da_visit(cand_off, n_poles, lb, ub, seed, t, pop: Population, qv=DA_QV, t0=DA_T0):
    """Proposals of generation t into pop.u."""
    cand_off = np.ascontiguousarray(cand_off, np.int64)
    n_poles = np.ascontiguousarray(n_poles, np.int32)
    lib().orc_da_visit(len(n_poles), _p(cand_off, _i64), _p(n_poles, _i32), pop.x.shape[1], _p(_f64(lb), _d),
                       _p(_f64(ub), _d), qv, t0, seed, t, _p(pop.x, _d), _p(pop.u, _d))


def da_accept(cand_off, n_poles, seed, t, u, cost_u, pop: Population, qv=DA_QV, qa=DA_QA, t0=DA_T0):
    cand_off = np.ascontiguousarray(cand_off, np.int64)
    n_poles = np.ascontiguousarray(n_poles, np.int32)
    u, cost_u = _f64(u), _f64(cost_u)
    lib().orc_da_accept(len(n_poles), _p(cand_off, _i64), _p(n_poles, _i32), pop.x.shape[1], qv, qa, t0, seed, t,
                        _p(u, _d), _p(cost_u, _d), _p(pop.x, _d), _p(pop.fit, _d), _p(pop.best_x, _d),
                        _p(pop.best_cost, _d), _p(pop.best_idx, _i64), _p(pop.history, _d), pop.history.shape[1])


def da_run(b: Batch, lb, ub, iters, seed=0, qv=DA_QV, qa=DA_QA, t0=DA_T0, ld=None, damping=1e-8, flags=0,
           nthreads=0):
    """Whole annealing: chains initialised in the box (generation 0), then
    `iters` x (propose, evaluate, accept).  P*(iters+1) evaluations."""
    ld = ld or int(b.n_poles.max())
    pop = Population(b.P, b.M, ld, iters + 1)
    da_init(b.cand_off, b.n_poles, lb, ub, seed, pop)
    da_accept(b.cand_off, b.n_poles, seed, 0, pop.x.copy(), fit_eval(b, pop.x, damping, flags, nthreads=nthreads)[0],
              pop, qv, qa, t0)
    for t in range(1, iters + 1):
        da_visit(b.cand_off, b.n_poles, lb, ub, seed, t, pop, qv, t0)
        da_accept(b.cand_off, b.n_poles, seed, t, pop.u, fit_eval(b, pop.u, damping, flags, nthreads=nthreads)[0],
                  pop, qv, qa, t0)
    return pop
