"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module holds no arithmetic of the fitting method: it only draws material
parameters, frequency grids, candidate log10(tau) batches and the batch layout
(offsets).  Target spectra are computed from these parameters by each side's
own material model.

The paper fits a Havriliak-Negami example (Sec. IV: 10 MHz-100 GHz, N = 5) and
names HN, Cole-Cole, Cole-Davidson, Jonscher, CRIM and user-tabulated data
(Sec. II-B, Sec. III-A).  It ships no dataset; the workloads below are seeded
stand-ins with those material families, frequency bands, pole counts and swarm
sizes.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

KIND_DEBYE, KIND_HN, KIND_CC, KIND_CD, KIND_JONSCHER, KIND_CRIM, KIND_HNSUM = range(7)
PARAM_STRIDE = 16
KIND_NAMES = ["debye", "hn", "cole-cole", "cole-davidson", "jonscher", "crim", "hn-sum-table"]

# CRIM water phase (Debye): eps_inf, d_eps, tau (s)
WATER = (4.9, 75.0, 9.2e-12)


def rng(seed: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[int(seed), int(stream)]))


def log_grid(fmin: float, fmax: float, F: int) -> np.ndarray:
    """Angular frequencies 2*pi*f on F log-spaced points, endpoints included."""
    return 2.0 * np.pi * np.logspace(math.log10(fmin), math.log10(fmax), F)


def tau_bounds(fmin: float, fmax: float) -> tuple[float, float]:
    """Search box for log10(tau): one decade beyond the fastest relaxation the
    band resolves, up to the slowest one."""
    lb = math.floor(-math.log10(2 * math.pi * fmax)) - 1
    ub = math.floor(-math.log10(2 * math.pi * fmin))
    return float(lb), float(ub)


def offsets(sizes) -> np.ndarray:
    o = np.zeros(len(sizes) + 1, dtype=np.int64)
    o[1:] = np.cumsum(np.asarray(sizes, dtype=np.int64))
    return o


# ---------------------------------------------------------------------------
# material parameter draws (rows of PARAM_STRIDE doubles)
# ---------------------------------------------------------------------------
def hn_params(eps_inf, d_eps, tau0, alpha, beta):
    p = np.zeros(PARAM_STRIDE)
    p[:5] = [eps_inf, d_eps, tau0, alpha, beta]
    return p


def draw_mixed(M: int, seed: int, fmin: float, fmax: float, kinds=None):
    """Mixed materials: kind uniform over HN / Cole-Cole / Cole-Davidson /
    Jonscher / CRIM (or over `kinds`).
    HN-family: eps_inf ~ U[2,8], d_eps ~ U[5,80], log10 tau0 ~ U[-11,-7],
    alpha, beta ~ U[0.3,1] (Cole-Cole beta = 1, Cole-Davidson alpha = 1).
    Jonscher eps_inf + chi (j w/w_p)^(n-1): n ~ U[0.1,0.9], chi ~ U[1,20],
    eps_inf ~ U[2,8], w_p = 2 pi sqrt(fmin fmax).
    CRIM: Debye water (4.9, 75, 9.2 ps) at volume fraction ~ U[0.05,0.4] in a
    lossless matrix eps_m ~ U[4,9]."""
    g = rng(seed, 1)
    kinds = [KIND_HN, KIND_CC, KIND_CD, KIND_JONSCHER, KIND_CRIM] if kinds is None else list(kinds)
    kind = np.asarray(kinds, dtype=np.int8)[g.integers(0, len(kinds), size=M)]
    u = g.random((M, 8))
    params = np.zeros((M, PARAM_STRIDE))
    for m in range(M):
        k = int(kind[m])
        if k in (KIND_HN, KIND_CC, KIND_CD, KIND_DEBYE):
            a = 0.3 + 0.7 * u[m, 3]
            b = 0.3 + 0.7 * u[m, 4]
            if k == KIND_CC:
                b = 1.0
            if k == KIND_CD:
                a = 1.0
            if k == KIND_DEBYE:
                a = b = 1.0
            params[m] = hn_params(2 + 6 * u[m, 0], 5 + 75 * u[m, 1], 10 ** (-11 + 4 * u[m, 2]), a, b)
        elif k == KIND_JONSCHER:
            params[m, :4] = [2 + 6 * u[m, 0], 1 + 19 * u[m, 1], 2 * math.pi * math.sqrt(fmin * fmax),
                             0.1 + 0.8 * u[m, 2]]
        elif k == KIND_CRIM:
            params[m, :5] = [WATER[0], WATER[1], WATER[2], 0.05 + 0.35 * u[m, 0], 4 + 5 * u[m, 1]]
        else:
            raise ValueError(k)
    return kind, params


def draw_hnsum(M: int, seed: int, noise: float = 0.01):
    """User-style tables: eps_inf ~ U[2,8] plus 1-3 HN terms (each drawn as in
    draw_mixed), with multiplicative Gaussian noise of relative size `noise`
    applied by the material model (Philox noise stream keyed by material)."""
    g = rng(seed, 2)
    kind = np.full(M, KIND_HNSUM, dtype=np.int8)
    params = np.zeros((M, PARAM_STRIDE))
    nt = g.integers(1, 4, size=M)
    u = g.random((M, 13))
    for m in range(M):
        params[m, 0] = 2 + 6 * u[m, 0]
        params[m, 1] = nt[m]
        for t in range(3):
            base = 2 + 4 * t
            if t < nt[m]:
                params[m, base:base + 4] = [5 + 75 * u[m, 1 + 4 * t], 10 ** (-11 + 4 * u[m, 2 + 4 * t]),
                                            0.3 + 0.7 * u[m, 3 + 4 * t], 0.3 + 0.7 * u[m, 4 + 4 * t]]
        params[m, 14] = noise
    return kind, params


def draw_theta(cand_off, n_poles, lb, ub, ld, seed: int) -> np.ndarray:
    """Candidate log10(tau) rows, uniform in each material's box; unused
    trailing columns are NaN."""
    g = rng(seed, 3)
    P = int(cand_off[-1])
    th = np.full((P, ld), np.nan)
    for m in range(len(n_poles)):
        a, b = int(cand_off[m]), int(cand_off[m + 1])
        N = int(n_poles[m])
        th[a:b, :N] = lb[m] + (ub[m] - lb[m]) * g.random((b - a, N))
    return th


# ---------------------------------------------------------------------------
# workload descriptions
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    kind: np.ndarray          # [M] int8
    params: np.ndarray        # [M][16]
    f_off: np.ndarray         # [M+1]
    omega: np.ndarray         # [F_tot]
    n_poles: np.ndarray       # [M] int32
    cand_off: np.ndarray      # [M+1]
    lb: np.ndarray            # [M]
    ub: np.ndarray            # [M]
    iters: int
    inertia: float = 0.7
    c1: float = 1.5
    c2: float = 1.5
    seed: int = 0
    polish_steps: int = 0
    noise_seed: int = 0

    @property
    def M(self):
        return len(self.n_poles)

    @property
    def P(self):
        return int(self.cand_off[-1])

    @property
    def ld(self):
        return int(self.n_poles.max())

    def evals(self):
        return self.P * (self.iters + 1)


def _uniform(name, kind, params, F, fmin, fmax, N, P, iters, **kw):
    M = len(kind)
    lb, ub = tau_bounds(fmin, fmax)
    om = log_grid(fmin, fmax, F)
    return Workload(name, kind, params, offsets([F] * M), np.tile(om, M), np.full(M, N, np.int32),
                    offsets([P] * M), np.full(M, lb), np.full(M, ub), iters, **kw)


def single_hn(seed: int = 0) -> Workload:
    """One HN material (eps_inf 3.4, d_eps 15, tau0 1 ns, a 0.8, b 0.6), F = 50
    on 1e5-1e10 Hz, N = 5, log10 tau in [-12, -6], 40 particles x 50 iterations."""
    kind = np.array([KIND_HN], np.int8)
    params = hn_params(3.4, 15.0, 1e-9, 0.8, 0.6)[None, :]
    return _uniform("single-hn F50 N5 P40 I50", kind, params, 50, 1e5, 1e10, 5, 40, 50, seed=seed)


def mixed_uniform(M=1024, F=1000, N=8, P=256, iters=200, seed: int = 0) -> Workload:
    """Mixed HN/CC/CD/Jonscher/CRIM materials on one 1e6-1e10 Hz grid."""
    kind, params = draw_mixed(M, seed, 1e6, 1e10)
    return _uniform(f"mixed M{M} F{F} N{N} P{P} I{iters}", kind, params, F, 1e6, 1e10, N, P, iters, seed=seed)


def mixed_ragged(M=4096, iters=300, seed: int = 0, fmax_points=5000, nmax=20) -> Workload:
    """Uneven batch: per material F ~ U{100..5000}, N ~ U{2..20}, swarm size in
    {64,128,256,512}, each with its own log grid on 1e6-1e10 Hz."""
    kind, params = draw_mixed(M, seed, 1e6, 1e10)
    g = rng(seed, 4)
    Fm = g.integers(100, fmax_points + 1, size=M)
    Nm = g.integers(2, nmax + 1, size=M).astype(np.int32)
    Pm = np.array([64, 128, 256, 512])[g.integers(0, 4, size=M)]
    lb, ub = tau_bounds(1e6, 1e10)
    omega = np.concatenate([log_grid(1e6, 1e10, int(f)) for f in Fm])
    return Workload(f"mixed-ragged M{M} I{iters}", kind, params, offsets(Fm), omega, Nm, offsets(Pm),
                    np.full(M, lb), np.full(M, ub), iters, seed=seed)


def hn_cc(M=1024, F=2000, N=12, P=256, iters=200, polish=50, seed: int = 0) -> Workload:
    """HN and Cole-Cole (50/50) on 1e5-1e11 Hz, with gradient polishing."""
    kind, params = draw_mixed(M, seed, 1e5, 1e11, kinds=[KIND_HN, KIND_CC])
    return _uniform(f"hn-cc M{M} F{F} N{N} P{P} I{iters} polish{polish}", kind, params, F, 1e5, 1e11, N, P,
                    iters, seed=seed, polish_steps=polish)


def tables(M=65536, F=4096, N=20, P=128, iters=400, polish=50, seed: int = 0) -> Workload:
    """Tabulated materials (1-3 HN terms + 1% noise) on 1e5-1e11 Hz."""
    kind, params = draw_hnsum(M, seed)
    return _uniform(f"tables M{M} F{F} N{N} P{P} I{iters} polish{polish}", kind, params, F, 1e5, 1e11, N, P,
                    iters, seed=seed, polish_steps=polish, noise_seed=seed + 17)
