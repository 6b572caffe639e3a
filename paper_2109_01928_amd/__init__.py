"""Python binding of the MI355X (gfx950) Debye fitting library.

Majchrowska et al., "Modelling Arbitrary Complex Dielectric Properties - an
automated implementation for gprMax": the multi-pole Debye expansion (Eq. 7)
is fitted by a hybrid scheme (Sec. III-B) - a swarm optimiser over the
relaxation times and a damped least-squares solve for the weights - here run
for thousands of materials at once on one GPU.

Every computation runs in the hand-written HIP kernels of ``libdebyefit.so``
(C ABI in ``include/debyefit.h``).  This module only marshals torch device
tensors (memory) and the current torch stream into those calls; it has no
CPU fallback and raises if the library is missing.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdebyefit.so")

OK, EINVAL, ERANGE, EHIP, ENOMEM = 0, -1, -2, -3, -4
ST_OK, ST_BADINPUT, ST_SINGULAR = 0, 1, 2
FLAG_NO_SIGN_FLIP = 1
FLAG_NO_REFINE = 2
FLAG_DD_REFINE = 4
PLAN_TARGET_GRAD = 1
LAUNCH_AUTO, LAUNCH_BUCKETS, LAUNCH_PERSISTENT = 0, 1, 2
MAX_POLES = 24
PARAM_STRIDE = 16
DEFAULT_DAMPING = 1e-8

EXPORTED = ["debye_plan_create", "debye_plan_destroy", "debye_plan_set_freq_split", "debye_plan_autotune",
            "debye_plan_set_launch", "debye_plan_get_launch",
            "debye_schedule_preview",
            "debye_plan_info",
            "debye_last_error", "debye_version", "debye_basis", "debye_fit_eval", "debye_fit_eval_grad",
            "debye_fit_eval_grad_noalloc",
            "debye_material_eval", "debye_material_vjp", "debye_pso_init", "debye_pso_step",
            "debye_pso_run", "debye_afe", "debye_fit_auto", "debye_de_init", "debye_de_trial", "debye_de_select", "debye_de_run",
            "debye_da_init", "debye_da_visit", "debye_da_accept", "debye_da_run", "debye_polish_create",
            "debye_polish_destroy", "debye_polish_begin", "debye_polish_step", "debye_lbfgs_polish"]


class DebyeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"debyefit error {code}: {msg}")
        self.code = code


class _CBatch(C.Structure):
    _fields_ = [("n_mat", C.c_int32), ("max_poles", C.c_int32), ("n_freq", C.c_int64), ("n_cand", C.c_int64),
                ("f_off", C.c_void_p), ("cand_off", C.c_void_p), ("n_poles", C.c_void_p),
                ("omega", C.c_void_p), ("eps_re", C.c_void_p), ("eps_im", C.c_void_p)]


class _CPso(C.Structure):
    _fields_ = [("inertia", C.c_double), ("c1", C.c_double), ("c2", C.c_double), ("seed", C.c_uint64)]


class _CSwarm(C.Structure):
    _fields_ = [("x", C.c_void_p), ("v", C.c_void_p), ("pbest_x", C.c_void_p), ("pbest_cost", C.c_void_p),
                ("gbest_x", C.c_void_p), ("gbest_cost", C.c_void_p), ("gbest_idx", C.c_void_p),
                ("history", C.c_void_p), ("hist_ld", C.c_int64), ("cost", C.c_void_p), ("status", C.c_void_p)]


class _CDe(C.Structure):
    _fields_ = [("f_lo", C.c_double), ("f_hi", C.c_double), ("cr", C.c_double), ("seed", C.c_uint64)]


class _CDa(C.Structure):
    _fields_ = [("qv", C.c_double), ("qa", C.c_double), ("t0", C.c_double), ("seed", C.c_uint64)]


class _CPop(C.Structure):
    _fields_ = [("x", C.c_void_p), ("u", C.c_void_p), ("fit", C.c_void_p), ("cost", C.c_void_p),
                ("best_x", C.c_void_p), ("best_cost", C.c_void_p), ("best_idx", C.c_void_p),
                ("history", C.c_void_p), ("hist_ld", C.c_int64), ("status", C.c_void_p)]


class _CAuto(C.Structure):
    _fields_ = [("n_min", C.c_int32), ("n_max", C.c_int32), ("chunk", C.c_int32), ("afe_target", C.c_double),
                ("particles", C.c_int32), ("iters", C.c_int32), ("pso", _CPso), ("polish_steps", C.c_int32)]


class _CLbfgs(C.Structure):
    _fields_ = [("steps", C.c_int32), ("mem", C.c_int32), ("max_trials", C.c_int32), ("c1", C.c_double)]


_lib = None
_vp = C.c_void_p


def lib():
    """Load libdebyefit.so (built in-tree by paper_2109_01928_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    i32, i64, dbl, u32 = C.c_int32, C.c_int64, C.c_double, C.c_uint32
    L.debye_last_error.restype = C.c_char_p
    L.debye_version.restype = C.c_char_p
    L.debye_plan_create.argtypes = [C.POINTER(_CBatch), _vp, _vp, _vp, u32, C.POINTER(_vp)]
    L.debye_plan_destroy.argtypes = [_vp]
    L.debye_plan_set_freq_split.argtypes = [_vp, i32, i32]
    L.debye_plan_set_launch.argtypes = [_vp, i32]
    L.debye_plan_get_launch.argtypes = [_vp]
    L.debye_plan_info.argtypes = [_vp, i32, _vp, _vp, _vp, _vp, _vp]
    L.debye_plan_autotune.argtypes = [_vp, C.POINTER(_CBatch), _vp, i64, dbl, u32, i32, _vp]
    L.debye_schedule_preview.argtypes = [_vp, _vp, _vp, i32, i32, i32, i32, _vp, _vp, i64, _vp, _vp]
    L.debye_basis.argtypes = [_vp, i64, _vp, i64, i64, i32, _vp, _vp, _vp]
    L.debye_fit_eval.argtypes = [_vp, C.POINTER(_CBatch), _vp, i64, dbl, u32, _vp, _vp, _vp, _vp, _vp]
    L.debye_fit_eval_grad.argtypes = [_vp, C.POINTER(_CBatch), _vp, i64, dbl, u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.debye_fit_eval_grad_noalloc.argtypes = L.debye_fit_eval_grad.argtypes
    L.debye_material_eval.argtypes = [i32, _vp, _vp, _vp, i64, _vp, C.c_uint64, _vp, _vp, _vp, _vp]
    L.debye_material_vjp.argtypes = [i32, _vp, i64, _vp, _vp, _vp, _vp, _vp]
    L.debye_pso_init.argtypes = [C.POINTER(_CBatch), i64, _vp, _vp, _CPso, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.debye_pso_step.argtypes = [C.POINTER(_CBatch), i64, _vp, _vp, _CPso, i32, i32, _vp, _vp, _vp, _vp, _vp, _vp,
                                 _vp, _vp, _vp, i64, _vp]
    L.debye_pso_run.argtypes = [_vp, C.POINTER(_CBatch), i64, _vp, _vp, _CPso, i32, dbl, u32, C.POINTER(_CSwarm), i32,
                                _vp]
    L.debye_afe.argtypes = [C.POINTER(_CBatch), _vp, i64, _vp, _vp, _vp, _vp]
    L.debye_fit_auto.argtypes = [C.POINTER(_CBatch), _vp, _vp, _vp, _CAuto, dbl, u32, _vp, _vp, _vp, _vp, _vp, i64,
                                 _vp]
    L.debye_de_init.argtypes = [C.POINTER(_CBatch), i64, _vp, _vp, _CDe, _vp, _vp, _vp, _vp, _vp]
    L.debye_de_trial.argtypes = [C.POINTER(_CBatch), i64, _vp, _vp, _CDe, i32, _vp, _vp, _vp]
    L.debye_de_select.argtypes = [C.POINTER(_CBatch), i64, i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, i64, _vp]
    L.debye_de_run.argtypes = [_vp, C.POINTER(_CBatch), i64, _vp, _vp, _CDe, i32, dbl, u32, C.POINTER(_CPop), i32, _vp]
    L.debye_da_init.argtypes = [C.POINTER(_CBatch), i64, _vp, _vp, _CDa, _vp, _vp, _vp, _vp, _vp]
    L.debye_da_visit.argtypes = [C.POINTER(_CBatch), i64, _vp, _vp, _CDa, i32, _vp, _vp, _vp]
    L.debye_da_accept.argtypes = [C.POINTER(_CBatch), i64, _CDa, i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, i64, _vp]
    L.debye_da_run.argtypes = [_vp, C.POINTER(_CBatch), i64, _vp, _vp, _CDa, i32, dbl, u32, C.POINTER(_CPop), i32, _vp]
    L.debye_polish_create.argtypes = [C.POINTER(_CBatch), _vp, _vp, i64, _CLbfgs, C.POINTER(_vp)]
    L.debye_polish_destroy.argtypes = [_vp]
    L.debye_polish_begin.argtypes = [_vp, C.POINTER(_CBatch), _vp, dbl, u32, _vp]
    L.debye_polish_step.argtypes = [_vp, C.POINTER(_CBatch), _vp, _vp, _vp, dbl, u32, i32, _vp, _vp]
    L.debye_lbfgs_polish.argtypes = [_vp, C.POINTER(_CBatch), _vp, _vp, _vp, dbl, u32, _vp, _vp]
    _lib = L
    return L


def _check(rc):
    if rc != OK:
        raise DebyeError(rc, lib().debye_last_error().decode())


def _ptr(t):
    return None if t is None else _vp(t.data_ptr())


def _stream():
    return _vp(torch.cuda.current_stream().cuda_stream)


def _dev(x, dtype, device):
    return torch.as_tensor(np.asarray(x), dtype=dtype).to(device).contiguous()


# ---------------------------------------------------------------------------
class Batch:
    """A ragged batch resident on the GPU: material m owns frequency points
    f_off[m]:f_off[m+1] and candidates cand_off[m]:cand_off[m+1] and is fitted
    with n_poles[m] poles.  Host copies of the shape are kept for planning."""

    def __init__(self, f_off, cand_off, n_poles, omega, eps_re, eps_im, device="cuda"):
        self.f_off_h = np.ascontiguousarray(np.asarray(f_off, dtype=np.int64))
        self.cand_off_h = np.ascontiguousarray(np.asarray(cand_off, dtype=np.int64))
        self.n_poles_h = np.ascontiguousarray(np.asarray(n_poles, dtype=np.int32))
        self.device = device
        self.f_off = _dev(self.f_off_h, torch.int64, device)
        self.cand_off = _dev(self.cand_off_h, torch.int64, device)
        self.n_poles = _dev(self.n_poles_h, torch.int32, device)
        self.omega = omega if torch.is_tensor(omega) else _dev(omega, torch.float64, device)
        self.eps_re = eps_re if torch.is_tensor(eps_re) else _dev(eps_re, torch.float64, device)
        self.eps_im = eps_im if torch.is_tensor(eps_im) else _dev(eps_im, torch.float64, device)
        self.M = len(self.n_poles_h)
        self.P = int(self.cand_off_h[-1])
        self.F = int(self.f_off_h[-1])
        self.max_poles = int(self.n_poles_h.max())

    def cstruct(self):
        for t in (self.omega, self.eps_re, self.eps_im):
            assert t.dtype == torch.float64 and t.is_contiguous() and t.numel() == self.F
        return _CBatch(self.M, self.max_poles, self.F, self.P, self.f_off.data_ptr(), self.cand_off.data_ptr(),
                       self.n_poles.data_ptr(), self.omega.data_ptr(), self.eps_re.data_ptr(), self.eps_im.data_ptr())

    def with_targets(self, eps_re, eps_im):
        b = object.__new__(Batch)
        b.__dict__.update(self.__dict__)
        b.eps_re, b.eps_im = eps_re.contiguous(), eps_im.contiguous()
        return b


def schedule_preview(f_off, cand_off, mats, n_poles, pole_split, freq_split):
    """Host-only preview of a bucket's work tiles (debye_schedule_preview):
    (lane_cand, lane_mat, xcd_off, uniform); no GPU needed."""
    f_off = np.ascontiguousarray(f_off, np.int64)
    cand_off = np.ascontiguousarray(cand_off, np.int64)
    mats = np.ascontiguousarray(mats, np.int32)
    xo = np.zeros(9, np.int64)
    uni = C.c_int32()
    p = lambda a: a.ctypes.data_as(_vp)
    n = lib().debye_schedule_preview(p(f_off), p(cand_off), p(mats), len(mats), n_poles, pole_split, freq_split,
                                     None, None, 0, p(xo), C.byref(uni))
    if n < 0:
        _check(n)
    lc = np.empty(n, np.int32)
    lm = np.empty(n, np.int32)
    _check(min(0, lib().debye_schedule_preview(p(f_off), p(cand_off), p(mats), len(mats), n_poles, pole_split,
                                               freq_split, p(lc), p(lm), n, p(xo), C.byref(uni))))
    return lc, lm, xo, bool(uni.value)


class Plan:
    """Launch schedule for one batch shape (see debye_plan_create).  With
    target_grads the plan also holds the adjoint records that target gradients
    (fit_eval_grad(..., targets=True), DebyeCost with eps gradients) need."""

    def __init__(self, b: Batch, target_grads=False):
        self.handle = _vp()
        self.target_grads = bool(target_grads)
        cb = b.cstruct()
        _check(lib().debye_plan_create(C.byref(cb), b.f_off_h.ctypes.data_as(_vp), b.cand_off_h.ctypes.data_as(_vp),
                                       b.n_poles_h.ctypes.data_as(_vp), PLAN_TARGET_GRAD if target_grads else 0,
                                       C.byref(self.handle)))

    def set_freq_split(self, split, n_poles=0):
        _check(lib().debye_plan_set_freq_split(self.handle, n_poles, split))

    def set_launch(self, mode):
        """LAUNCH_BUCKETS (per-bucket launches), LAUNCH_PERSISTENT (one
        persistent launch over every bucket) or LAUNCH_AUTO (debye_plan_set_launch)."""
        _check(lib().debye_plan_set_launch(self.handle, int(mode)))

    def launch(self):
        rc = lib().debye_plan_get_launch(self.handle)
        if rc < 0:
            _check(rc)
        return rc

    def autotune(self, b: "Batch", theta, damping=1e-8, flags=0, reps=3):
        """Time each bucket's frequency splits on (b, theta) and keep the fastest
        (debye_plan_autotune; synchronises the current stream)."""
        assert theta.dtype == torch.float64 and theta.is_contiguous() and theta.dim() == 2 and theta.shape[0] == b.P
        cb = b.cstruct()
        _check(lib().debye_plan_autotune(self.handle, C.byref(cb), _ptr(theta), theta.shape[1], damping, flags, reps,
                                         _stream()))

    def info(self):
        L = lib()
        n = L.debye_plan_info(self.handle, -1, None, None, None, None, None)
        out = []
        for i in range(n):
            N, sp, sf, un = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
            nt = C.c_int64()
            _check(L.debye_plan_info(self.handle, i, C.byref(N), C.byref(sp), C.byref(sf), C.byref(nt), C.byref(un)))
            out.append(dict(n_poles=N.value, pole_split=sp.value, freq_split=sf.value, tiles=nt.value,
                            uniform=bool(un.value)))
        return out

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.debye_plan_destroy(self.handle)
            self.handle = None


# ---------------------------------------------------------------------------
def fit_eval(plan: Plan, b: Batch, theta, damping=DEFAULT_DAMPING, flags=0, want_weights=True, out=None):
    """Cost (and weights, eps_inf, status) of every candidate (debye_fit_eval)."""
    ld = theta.shape[1]
    P = b.P
    dev = theta.device
    if out is None:
        cost = torch.empty(P, dtype=torch.float64, device=dev)
        w = torch.empty((P, ld), dtype=torch.float64, device=dev) if want_weights else None
        einf = torch.empty(P, dtype=torch.float64, device=dev) if want_weights else None
        st = torch.empty(P, dtype=torch.int8, device=dev)
    else:
        cost, w, einf, st = out
    cb = b.cstruct()
    _check(lib().debye_fit_eval(plan.handle, C.byref(cb), _ptr(theta), ld, float(damping), flags, _ptr(cost), _ptr(w),
                                _ptr(einf), _ptr(st), _stream()))
    return cost, w, einf, st


def fit_eval_grad(plan: Plan, b: Batch, theta, damping=DEFAULT_DAMPING, flags=0, grad_cost=None, targets=False,
                  noalloc=False, out=None):
    """Cost and the variable-projection adjoint (debye_fit_eval_grad; with
    noalloc, debye_fit_eval_grad_noalloc: target-gradient records in the
    library's static workspace, no DEBYE_PLAN_TARGET_GRAD plan needed).
    `out` (cost, grad_theta, grad_re, grad_im, status) reuses tensors."""
    ld = theta.shape[1]
    dev = theta.device
    if out is None:
        cost = torch.empty(b.P, dtype=torch.float64, device=dev)
        g = torch.empty((b.P, ld), dtype=torch.float64, device=dev)
        st = torch.empty(b.P, dtype=torch.int8, device=dev)
        gr = torch.empty(b.F, dtype=torch.float64, device=dev) if targets else None
        gi = torch.empty(b.F, dtype=torch.float64, device=dev) if targets else None
    else:
        cost, g, gr, gi, st = out
    gc = None if grad_cost is None else grad_cost.to(torch.float64).contiguous()
    cb = b.cstruct()
    fn = lib().debye_fit_eval_grad_noalloc if noalloc else lib().debye_fit_eval_grad
    _check(fn(plan.handle, C.byref(cb), _ptr(theta), ld, float(damping), flags, _ptr(gc), _ptr(cost), _ptr(g),
              _ptr(gr), _ptr(gi), _ptr(st), _stream()))
    return cost, g, gr, gi, st


def material_eval(kind, params, b_or_f_off, omega=None, noise_seed=0, jac=False, device="cuda"):
    """Targets eps', eps'' (and the HN-family Jacobian) on the GPU (debye_material_eval)."""
    if isinstance(b_or_f_off, Batch):
        f_off, omega, F = b_or_f_off.f_off, b_or_f_off.omega, b_or_f_off.F
    else:
        f_off = _dev(b_or_f_off, torch.int64, device)
        F = int(np.asarray(b_or_f_off)[-1])
        omega = omega if torch.is_tensor(omega) else _dev(omega, torch.float64, device)
    kind_t = kind if torch.is_tensor(kind) else _dev(np.asarray(kind, np.int8), torch.int8, device)
    par = params if torch.is_tensor(params) else _dev(np.asarray(params, np.float64).reshape(-1, PARAM_STRIDE),
                                                      torch.float64, device)
    er = torch.empty(F, dtype=torch.float64, device=omega.device)
    ei = torch.empty(F, dtype=torch.float64, device=omega.device)
    J = torch.empty((F, 5, 2), dtype=torch.float64, device=omega.device) if jac else None
    _check(lib().debye_material_eval(len(kind_t), _ptr(kind_t), _ptr(par), _ptr(f_off), F, _ptr(omega),
                                     C.c_uint64(noise_seed), _ptr(er), _ptr(ei), _ptr(J), _stream()))
    return (er, ei, J) if jac else (er, ei)


def basis(omega, theta, N):
    """Debye basis re/im [n_cand][N][F] (debye_basis)."""
    F = omega.numel()
    n = theta.shape[0]
    re = torch.empty((n, N, F), dtype=torch.float64, device=omega.device)
    im = torch.empty_like(re)
    _check(lib().debye_basis(_ptr(omega), F, _ptr(theta), theta.shape[1], n, N, _ptr(re), _ptr(im), _stream()))
    return re, im


# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Swarm:
    x: torch.Tensor
    v: torch.Tensor
    pbest_x: torch.Tensor
    pbest_cost: torch.Tensor
    gbest_x: torch.Tensor
    gbest_cost: torch.Tensor
    gbest_idx: torch.Tensor
    history: torch.Tensor

    @staticmethod
    def empty(P, M, ld, hist_len, device="cuda"):
        f = dict(dtype=torch.float64, device=device)
        return Swarm(torch.zeros((P, ld), **f), torch.zeros((P, ld), **f), torch.zeros((P, ld), **f),
                     torch.zeros(P, **f), torch.zeros((M, ld), **f), torch.zeros(M, **f),
                     torch.zeros(M, dtype=torch.int64, device=device),
                     torch.full((M, max(hist_len, 1)), float("nan"), **f))


def pso_init(b: Batch, lb, ub, sw: Swarm, inertia=0.7, c1=1.5, c2=1.5, seed=0):
    cb = b.cstruct()
    p = _CPso(inertia, c1, c2, seed)
    _check(lib().debye_pso_init(C.byref(cb), sw.x.shape[1], _ptr(lb), _ptr(ub), p, _ptr(sw.x), _ptr(sw.v),
                                _ptr(sw.pbest_x), _ptr(sw.pbest_cost), _ptr(sw.gbest_cost), _ptr(sw.gbest_idx),
                                _stream()))


def pso_step(b: Batch, lb, ub, sw: Swarm, t, move, cost, inertia=0.7, c1=1.5, c2=1.5, seed=0, history=True):
    cb = b.cstruct()
    p = _CPso(inertia, c1, c2, seed)
    h = sw.history if history else None
    _check(lib().debye_pso_step(C.byref(cb), sw.x.shape[1], _ptr(lb), _ptr(ub), p, int(t), int(move), _ptr(cost),
                                _ptr(sw.x), _ptr(sw.v), _ptr(sw.pbest_x), _ptr(sw.pbest_cost), _ptr(sw.gbest_x),
                                _ptr(sw.gbest_cost), _ptr(sw.gbest_idx), _ptr(h), sw.history.shape[1], _stream()))


def pso_run(plan: Plan, b: Batch, lb, ub, sw: Swarm, iters, inertia=0.7, c1=1.5, c2=1.5, seed=0,
            damping=DEFAULT_DAMPING, flags=0, use_graph=True, cost=None, status=None):
    """A whole swarm fit (debye_pso_run); returns the cost of the final positions."""
    cost = torch.empty(b.P, dtype=torch.float64, device=sw.x.device) if cost is None else cost
    cs = _CSwarm(sw.x.data_ptr(), sw.v.data_ptr(), sw.pbest_x.data_ptr(), sw.pbest_cost.data_ptr(),
                 sw.gbest_x.data_ptr(), sw.gbest_cost.data_ptr(), sw.gbest_idx.data_ptr(), sw.history.data_ptr(),
                 sw.history.shape[1], cost.data_ptr(), None if status is None else status.data_ptr())
    cb = b.cstruct()
    _check(lib().debye_pso_run(plan.handle, C.byref(cb), sw.x.shape[1], _ptr(lb), _ptr(ub),
                               _CPso(inertia, c1, c2, seed), int(iters), float(damping), flags, C.byref(cs),
                               1 if use_graph else 0, _stream()))
    return cost


def afe(b: Batch, theta, weights, eps_inf):
    """Average fractional error (percent) of every candidate's fitted expansion (debye_afe)."""
    out = torch.empty(b.P, dtype=torch.float64, device=theta.device)
    cb = b.cstruct()
    _check(lib().debye_afe(C.byref(cb), _ptr(theta), theta.shape[1], _ptr(weights), _ptr(eps_inf), _ptr(out),
                           _stream()))
    return out


def fit_auto(b: Batch, lb, ub, n_min=1, n_max=20, chunk=4, afe_target=5.0, particles=64, iters=100,
             inertia=0.7, c1=1.5, c2=1.5, seed=0, polish_steps=20, damping=DEFAULT_DAMPING, flags=0):
    """Automatic pole count (debye_fit_auto): the smallest N in n_min..n_max whose
    fitted expansion has an average fractional error below afe_target percent.
    b describes the materials' spectra (its candidate fields are ignored).
    Returns (n_poles [M], log10_tau [M][n_max], weights [M][n_max], eps_inf [M], afe [M])."""
    dev = b.omega.device
    M = b.M
    n = torch.zeros(M, dtype=torch.int32, device=dev)
    th = torch.full((M, n_max), float("nan"), dtype=torch.float64, device=dev)
    w = torch.full((M, n_max), float("nan"), dtype=torch.float64, device=dev)
    einf = torch.empty(M, dtype=torch.float64, device=dev)
    err = torch.empty(M, dtype=torch.float64, device=dev)
    cb = b.cstruct()
    prm = _CAuto(n_min, n_max, chunk, afe_target, particles, iters, _CPso(inertia, c1, c2, seed), polish_steps)
    _check(lib().debye_fit_auto(C.byref(cb), b.f_off_h.ctypes.data_as(_vp), _ptr(lb), _ptr(ub), prm, float(damping),
                                flags, _ptr(n), _ptr(th), _ptr(w), _ptr(einf), _ptr(err), n_max, _stream()))
    return n, th, w, einf, err


@dataclasses.dataclass
class Population:
    """Differential-evolution state (see debye_population)."""
    x: torch.Tensor
    u: torch.Tensor
    fit: torch.Tensor
    cost: torch.Tensor
    best_x: torch.Tensor
    best_cost: torch.Tensor
    best_idx: torch.Tensor
    history: torch.Tensor

    @staticmethod
    def empty(P, M, ld, hist_len, device="cuda"):
        f = dict(dtype=torch.float64, device=device)
        return Population(torch.zeros((P, ld), **f), torch.zeros((P, ld), **f), torch.zeros(P, **f),
                          torch.zeros(P, **f), torch.zeros((M, ld), **f), torch.zeros(M, **f),
                          torch.zeros(M, dtype=torch.int64, device=device),
                          torch.full((M, max(hist_len, 1)), float("nan"), **f))


def de_init(b: Batch, lb, ub, pop: Population, f_lo=0.5, f_hi=1.0, cr=0.7, seed=0):
    cb = b.cstruct()
    _check(lib().debye_de_init(C.byref(cb), pop.x.shape[1], _ptr(lb), _ptr(ub), _CDe(f_lo, f_hi, cr, seed),
                               _ptr(pop.x), _ptr(pop.fit), _ptr(pop.best_cost), _ptr(pop.best_idx), _stream()))


def de_trial(b: Batch, lb, ub, pop: Population, t, f_lo=0.5, f_hi=1.0, cr=0.7, seed=0):
    """pop.u = trial vectors of generation t (debye_de_trial)."""
    cb = b.cstruct()
    _check(lib().debye_de_trial(C.byref(cb), pop.x.shape[1], _ptr(lb), _ptr(ub), _CDe(f_lo, f_hi, cr, seed), int(t),
                                _ptr(pop.x), _ptr(pop.u), _stream()))


def de_select(b: Batch, pop: Population, t, u, cost_u, history=True):
    """Greedy replacement by the trials u with costs cost_u (debye_de_select)."""
    cb = b.cstruct()
    h = pop.history if history else None
    _check(lib().debye_de_select(C.byref(cb), pop.x.shape[1], int(t), _ptr(u), _ptr(cost_u), _ptr(pop.x),
                                 _ptr(pop.fit), _ptr(pop.best_x), _ptr(pop.best_cost), _ptr(pop.best_idx), _ptr(h),
                                 pop.history.shape[1], _stream()))


def de_run(plan: Plan, b: Batch, lb, ub, pop: Population, iters, f_lo=0.5, f_hi=1.0, cr=0.7, seed=0,
           damping=DEFAULT_DAMPING, flags=0, use_graph=True, status=None):
    """A whole differential-evolution fit (debye_de_run)."""
    cp = _CPop(pop.x.data_ptr(), pop.u.data_ptr(), pop.fit.data_ptr(), pop.cost.data_ptr(), pop.best_x.data_ptr(),
               pop.best_cost.data_ptr(), pop.best_idx.data_ptr(), pop.history.data_ptr(), pop.history.shape[1],
               None if status is None else status.data_ptr())
    cb = b.cstruct()
    _check(lib().debye_de_run(plan.handle, C.byref(cb), pop.x.shape[1], _ptr(lb), _ptr(ub),
                              _CDe(f_lo, f_hi, cr, seed), int(iters), float(damping), flags, C.byref(cp),
                              1 if use_graph else 0, _stream()))


DA_QV, DA_QA, DA_T0 = 2.62, -5.0, 5230.0


def da_init(b: Batch, lb, ub, pop: Population, qv=DA_QV, qa=DA_QA, t0=DA_T0, seed=0):
    cb = b.cstruct()
    _check(lib().debye_da_init(C.byref(cb), pop.x.shape[1], _ptr(lb), _ptr(ub), _CDa(qv, qa, t0, seed), _ptr(pop.x),
                               _ptr(pop.fit), _ptr(pop.best_cost), _ptr(pop.best_idx), _stream()))


def da_visit(b: Batch, lb, ub, pop: Population, t, qv=DA_QV, qa=DA_QA, t0=DA_T0, seed=0):
    """pop.u = proposals of generation t (debye_da_visit)."""
    cb = b.cstruct()
    _check(lib().debye_da_visit(C.byref(cb), pop.x.shape[1], _ptr(lb), _ptr(ub), _CDa(qv, qa, t0, seed), int(t),
                                _ptr(pop.x), _ptr(pop.u), _stream()))


def da_accept(b: Batch, pop: Population, t, y, cost_y, qv=DA_QV, qa=DA_QA, t0=DA_T0, seed=0, history=True):
    cb = b.cstruct()
    h = pop.history if history else None
    _check(lib().debye_da_accept(C.byref(cb), pop.x.shape[1], _CDa(qv, qa, t0, seed), int(t), _ptr(y), _ptr(cost_y),
                                 _ptr(pop.x), _ptr(pop.fit), _ptr(pop.best_x), _ptr(pop.best_cost),
                                 _ptr(pop.best_idx), _ptr(h), pop.history.shape[1], _stream()))


def da_run(plan: Plan, b: Batch, lb, ub, pop: Population, iters, qv=DA_QV, qa=DA_QA, t0=DA_T0, seed=0,
           damping=DEFAULT_DAMPING, flags=0, use_graph=True, status=None):
    """A whole annealing fit (debye_da_run)."""
    cp = _CPop(pop.x.data_ptr(), pop.u.data_ptr(), pop.fit.data_ptr(), pop.cost.data_ptr(), pop.best_x.data_ptr(),
               pop.best_cost.data_ptr(), pop.best_idx.data_ptr(), pop.history.data_ptr(), pop.history.shape[1],
               None if status is None else status.data_ptr())
    cb = b.cstruct()
    _check(lib().debye_da_run(plan.handle, C.byref(cb), pop.x.shape[1], _ptr(lb), _ptr(ub), _CDa(qv, qa, t0, seed),
                              int(iters), float(damping), flags, C.byref(cp), 1 if use_graph else 0, _stream()))


class Polish:
    """L-BFGS polish context for one candidate per material (debye_polish_create):
    owns the history, the trial buffers and the evaluation plans, so that
    begin/step/run only enqueue work (no allocation, no synchronisation)."""

    def __init__(self, b1: Batch, ld, steps=50, mem=10, max_trials=30, c1=1e-4):
        self.handle = _vp()
        self.steps = int(steps)
        cb = b1.cstruct()
        _check(lib().debye_polish_create(C.byref(cb), b1.f_off_h.ctypes.data_as(_vp), b1.n_poles_h.ctypes.data_as(_vp),
                                         int(ld), _CLbfgs(steps, mem, max_trials, c1), C.byref(self.handle)))

    def begin(self, b1: Batch, theta, damping=DEFAULT_DAMPING, flags=0):
        cb = b1.cstruct()
        _check(lib().debye_polish_begin(self.handle, C.byref(cb), _ptr(theta), float(damping), flags, _stream()))

    def step(self, b1: Batch, theta, lb, ub, step, damping=DEFAULT_DAMPING, flags=0, cost_hist=None):
        cb = b1.cstruct()
        _check(lib().debye_polish_step(self.handle, C.byref(cb), _ptr(theta), _ptr(lb), _ptr(ub), float(damping), flags,
                                       int(step), _ptr(cost_hist), _stream()))

    def run(self, b1: Batch, theta, lb, ub, damping=DEFAULT_DAMPING, flags=0, cost_hist=None):
        cb = b1.cstruct()
        _check(lib().debye_lbfgs_polish(self.handle, C.byref(cb), _ptr(theta), _ptr(lb), _ptr(ub), float(damping),
                                        flags, _ptr(cost_hist), _stream()))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.debye_polish_destroy(self.handle)
            self.handle = None


def lbfgs_polish(b1: Batch, theta, lb, ub, steps=50, mem=10, max_trials=30, c1=1e-4, damping=DEFAULT_DAMPING,
                 flags=0, history=True, polish=None):
    """L-BFGS polish of one candidate per material (theta [M][ld], in place)
    inside the box [lb[m], ub[m]] (device tensors [M]).  Creates a Polish
    context unless one (made for `steps`) is passed; returns the cost history
    [M][steps+1] (or None)."""
    if polish is None:
        polish = Polish(b1, theta.shape[1], steps, mem, max_trials, c1)
    hist = torch.empty((b1.M, polish.steps + 1), dtype=torch.float64, device=theta.device) if history else None
    polish.run(b1, theta, lb, ub, damping, flags, hist)
    return hist


# ---------------------------------------------------------------------------
class DebyeCost(torch.autograd.Function):
    """cost[c] = C(theta[c], eps'[m(c)], eps''[m(c)]) with the adjoint of
    debye_fit_eval_grad as backward (gradients for theta, eps', eps'')."""

    @staticmethod
    def forward(ctx, theta, eps_re, eps_im, plan, batch, damping=DEFAULT_DAMPING, flags=0):
        if flags & FLAG_DD_REFINE:
            raise ValueError("FLAG_DD_REFINE is a forward-evaluation flag: the adjoint has no double-double form")
        b = batch.with_targets(eps_re.detach(), eps_im.detach())
        cost = fit_eval(plan, b, theta.detach().contiguous(), damping, flags, want_weights=False)[0]
        ctx.save_for_backward(theta, eps_re, eps_im)
        ctx.plan, ctx.batch, ctx.damping, ctx.flags = plan, batch, damping, flags
        return cost

    @staticmethod
    def backward(ctx, grad_cost):
        theta, eps_re, eps_im = ctx.saved_tensors
        b = ctx.batch.with_targets(eps_re.detach(), eps_im.detach())
        want_t = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
        if want_t and not getattr(ctx.plan, "target_grads", False):
            raise ValueError("gradients for eps', eps'' need a Plan(batch, target_grads=True)")
        _, g, gr, gi, _ = fit_eval_grad(ctx.plan, b, theta.detach().contiguous(), ctx.damping, ctx.flags,
                                        grad_cost=grad_cost.contiguous(), targets=want_t)
        return g, gr, gi, None, None, None, None


class HNTarget(torch.autograd.Function):
    """Havriliak-Negami-family targets (Eq. 4) from params [M][16] with the
    analytic Jacobian of debye_material_eval as backward (columns eps_inf,
    d_eps, tau0, alpha, beta)."""

    @staticmethod
    def forward(ctx, params, kind, batch):
        er, ei, J = material_eval(kind, params.detach().contiguous(), batch, jac=True)
        ctx.save_for_backward(J)
        ctx.f_off = batch.f_off
        ctx.M = params.shape[0]
        return er, ei

    @staticmethod
    def backward(ctx, g_re, g_im):
        (J,) = ctx.saved_tensors
        return material_vjp(ctx.f_off, J, g_re, g_im, ctx.M), None, None


def material_vjp(f_off, jac, g_re, g_im, M):
    """Material-parameter gradient from the target gradients (debye_material_vjp)."""
    gp = torch.empty((M, PARAM_STRIDE), dtype=torch.float64, device=jac.device)
    _check(lib().debye_material_vjp(M, _ptr(f_off), jac.shape[0], _ptr(jac), _ptr(g_re.contiguous()),
                                    _ptr(g_im.contiguous()), _ptr(gp), _stream()))
    return gp
