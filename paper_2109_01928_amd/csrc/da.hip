// Annealing over log10(tau) (the paper's DA-DLS alternative, Sec. III-A):
// generalized simulated annealing (Tsallis & Stariolo 1996) as in dual
// annealing, batched: the candidates of a material are independent Markov
// chains.  Generation t >= 1:
//   visiting temperature   T(t) = T0 (2^(qv-1) - 1) / ((1 + t)^(qv-1) - 1)
//   acceptance temperature Ta(t) = T(t) / t
//   proposal  y_d = x_d + s(t) g_d, s(t) = T(t)^(1/(3-qv)) / sqrt(3 - qv),
//             g_d Student-t with nu = (3 - qv)/(qv - 1) (the one-dimensional
//             visiting distribution) by Bailey's polar method, wrapped
//             periodically into [lb, ub]
//   accept    if f(y) < f(x); else when z = 1 - (1 - qa)(f(y) - f(x))/Ta > 0
//             and u^(1-qa) < z
// Random numbers: Philox4x64-10, key (seed, material):
//   initial chain i, coordinate d:  counter (d, i, 0, DA_INIT), word 0
//   proposal coordinate d:          counter (d, i, t, DA_VISIT + 16 j), word
//                                   pairs (0,1), (2,3) for polar round j < 16
//   acceptance of chain i:          counter (0, i, t, DA_ACCEPT), word 0
// exp and log are evaluated from their series with every operation rounded
// on its own (no fused multiply-add), so that a run is bit-reproducible by any
// IEEE double implementation of the same steps.

#include <algorithm>

#include "common.hpp"
#include "rng.hpp"
#include "fit_eval.hpp"

namespace dfit {

namespace {

#pragma clang fp contract(off)

// ln 2 as a 20-bit head (k * head is exact) and the rest
constexpr double LN2_HEAD = 0x1.62e42p-1, LN2_TAIL = 0x1.fdf473de6af28p-22;
constexpr double INV_LN2 = 0x1.71547652b82fep+0;

// e^x: x = k ln2 + r (Cody & Waite reduction), e^r from the nested Taylor
// polynomial 1 + r (1 + r/2 (1 + ... (1 + r/17))), times 2^k
__device__ double sexp(double x) {
  if (x != x) return x;
  if (x > 709.0) return INFINITY;
  if (x < -745.0) return 0.0;
  const double k = __builtin_rint(__dmul_rn(x, INV_LN2));
  const double r = __dsub_rn(__dsub_rn(x, __dmul_rn(k, LN2_HEAD)), __dmul_rn(k, LN2_TAIL));
  double p = 1.0;
  for (int n = 17; n >= 1; --n) p = __dadd_rn(1.0, __dmul_rn(__ddiv_rn(r, (double)n), p));
  return ldexp(p, (int)k);
}

// log x: x = m 2^e, m in [sqrt(1/2), sqrt(2)), log m = 2 atanh((m-1)/(m+1))
// from its odd series to the 25th power
__device__ double slog(double x) {
  if (x != x || x < 0.0) return NAN;
  if (x == 0.0) return -INFINITY;
  if (x == INFINITY) return INFINITY;
  int e = 0;
  double m = frexp(x, &e);
  if (m < 0x1.6a09e667f3bcdp-1) {
    m = __dmul_rn(2.0, m);
    e -= 1;
  }
  const double s = __ddiv_rn(__dsub_rn(m, 1.0), __dadd_rn(m, 1.0));
  const double z = __dmul_rn(s, s);
  double q = __ddiv_rn(1.0, 25.0);
  for (int k = 11; k >= 0; --k) q = __dadd_rn(__dmul_rn(q, z), __ddiv_rn(1.0, (double)(2 * k + 1)));
  const double lm = __dmul_rn(__dmul_rn(2.0, s), q);
  return __dadd_rn(__dmul_rn((double)e, LN2_HEAD), __dadd_rn(__dmul_rn((double)e, LN2_TAIL), lm));
}

struct Temps {
  double visit_scale, accept_temp;
};

__device__ Temps temps(double qv, double t0, int32_t t) {
  const double a = __dsub_rn(qv, 1.0);
  const double num = __dsub_rn(sexp(__dmul_rn(a, slog(2.0))), 1.0);
  const double den = __dsub_rn(sexp(__dmul_rn(a, slog(__dadd_rn(1.0, (double)t)))), 1.0);
  const double T = __ddiv_rn(__dmul_rn(t0, num), den);
  Temps r;
  r.visit_scale = __ddiv_rn(sexp(__ddiv_rn(slog(T), __dsub_rn(3.0, qv))), __dsqrt_rn(__dsub_rn(3.0, qv)));
  r.accept_temp = __ddiv_rn(T, (double)t);
  return r;
}

__device__ double student_t(uint64_t seed, uint64_t m, uint64_t d, uint64_t i, uint64_t t, double nu) {
  for (int j = 0; j < 16; ++j) {
    const U64x4 w = philox4x64(d, i, t, (uint64_t)(STREAM_DA_VISIT + 16 * j), seed, m);
    for (int h = 0; h < 2; ++h) {
      const double u = __dsub_rn(__dmul_rn(2.0, unit53(w.w[2 * h])), 1.0);
      const double v = __dsub_rn(__dmul_rn(2.0, unit53(w.w[2 * h + 1])), 1.0);
      const double W = __dadd_rn(__dmul_rn(u, u), __dmul_rn(v, v));
      if (W > 0.0 && W <= 1.0) {
        double q = sexp(__dmul_rn(__ddiv_rn(-2.0, nu), slog(W)));
        if (q > 1e300) q = 1e300;
        return __dmul_rn(u, __dsqrt_rn(__ddiv_rn(__dmul_rn(nu, __dsub_rn(q, 1.0)), W)));
      }
    }
  }
  return 0.0;
}

__device__ double wrap_box(double y, double lo, double hi) {
  if (y >= lo && y <= hi) return y;
  const double span = __dsub_rn(hi, lo);
  double r = fmod(__dsub_rn(y, lo), span);
  if (r < 0.0) r = __dadd_rn(r, span);
  return __dadd_rn(lo, r);
}

__device__ __forceinline__ int mat_of(const int64_t *off, int32_t M, int64_t c) {
  int lo = 0, hi = M - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace

__global__ __launch_bounds__(256) void da_init_kernel(const DaArgs a, int64_t n_cand) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < a.M) {
    a.best_cost[c] = INFINITY;
    a.best_idx[c] = -1;
  }
  if (c >= n_cand) return;
  const int m = mat_of(a.cand_off, a.M, c);
  const int64_t i = c - a.cand_off[m];
  const double lo = a.lb[m], span = __dsub_rn(a.ub[m], a.lb[m]);
  for (int d = 0; d < a.n_poles[m]; ++d) {
    const U64x4 r = philox4x64((uint64_t)d, (uint64_t)i, 0, STREAM_DA_INIT, a.seed, (uint64_t)m);
    a.x[c * a.ld + d] = __dadd_rn(lo, __dmul_rn(span, unit53(r.w[0])));
  }
  a.fit[c] = INFINITY;
}

// one thread per chain: its proposal
__global__ __launch_bounds__(256) void da_visit_kernel(const DaArgs a, int64_t n_cand) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cand) return;
  const int32_t t = a.t_dev ? *a.t_dev : a.t;
  const int m = mat_of(a.cand_off, a.M, c);
  const int64_t i = c - a.cand_off[m];
  const Temps tp = temps(a.qv, a.t0, t);
  const double nu = __ddiv_rn(__dsub_rn(3.0, a.qv), __dsub_rn(a.qv, 1.0));
  const double lo = a.lb[m], hi = a.ub[m];
  for (int d = 0; d < a.n_poles[m]; ++d) {
    const double g = student_t(a.seed, (uint64_t)m, (uint64_t)d, (uint64_t)i, (uint64_t)t, nu);
    a.u[c * a.ld + d] = wrap_box(__dadd_rn(a.x[c * a.ld + d], __dmul_rn(tp.visit_scale, g)), lo, hi);
  }
}

// one block per material: acceptance, then the best visited state
__global__ __launch_bounds__(256) void da_accept_kernel(const DaArgs a) {
  __shared__ double s_val[256];
  __shared__ int64_t s_idx[256];
  __shared__ int s_take;
  const int m = blockIdx.x;
  const int tid = threadIdx.x;
  const int32_t t = a.t_dev ? *a.t_dev : a.t;
  const int64_t c0 = a.cand_off[m];
  const int64_t P = a.cand_off[m + 1] - c0;
  const int N = a.n_poles[m];
  const int64_t ld = a.ld;
  const double ta = t > 0 ? temps(a.qv, a.t0, t).accept_temp : 0.0;
  for (int64_t p = tid; p < P; p += blockDim.x) {
    const int64_t c = c0 + p;
    const double fy = a.cost_u[c], fx = a.fit[c];
    bool take;
    if (t == 0 || fy < fx) {
      take = fy == fy;
    } else if (fy != fy) {
      take = false;
    } else {
      const double z = __dsub_rn(1.0, __ddiv_rn(__dmul_rn(__dsub_rn(1.0, a.qa), __dsub_rn(fy, fx)), ta));
      take = false;
      if (z > 0.0) {
        const U64x4 w = philox4x64(0, (uint64_t)p, (uint64_t)t, STREAM_DA_ACCEPT, a.seed, (uint64_t)m);
        take = sexp(__dmul_rn(__dsub_rn(1.0, a.qa), slog(unit53(w.w[0])))) < z;
      }
    }
    if (take) {
      a.fit[c] = fy;
      for (int d = 0; d < N; ++d) a.x[c * ld + d] = a.u[c * ld + d];
    }
  }
  __syncthreads();
  double bv = INFINITY;
  int64_t bi = -1;
  for (int64_t p = tid; p < P; p += blockDim.x) {
    const double f = a.fit[c0 + p];
    if (f == f && (bi < 0 || f < bv)) {
      bv = f;
      bi = p;
    }
  }
  s_val[tid] = bv;
  s_idx[tid] = bi;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w) {
      const double v2 = s_val[tid + w], v1 = s_val[tid];
      const int64_t i2 = s_idx[tid + w], i1 = s_idx[tid];
      if (i2 >= 0 && (i1 < 0 || v2 < v1 || (v2 == v1 && i2 < i1))) {
        s_val[tid] = v2;
        s_idx[tid] = i2;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int take = (s_idx[0] >= 0 && s_val[0] < a.best_cost[m]) ? 1 : 0;
    s_take = take;
    if (take) {
      a.best_cost[m] = s_val[0];
      a.best_idx[m] = s_idx[0];
    }
    if (a.history) a.history[(int64_t)m * a.hist_ld + t] = a.best_cost[m];
  }
  __syncthreads();
  if (s_take)
    for (int d = tid; d < N; d += blockDim.x) a.best_x[(int64_t)m * ld + d] = a.x[(c0 + s_idx[0]) * ld + d];
}

hipError_t launch_da_init(const DaArgs &a, int64_t n_cand, hipStream_t s) {
  const int64_t n = n_cand > a.M ? n_cand : a.M;
  hipLaunchKernelGGL(da_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, n_cand);
  return hipGetLastError();
}

hipError_t launch_da_visit(const DaArgs &a, int64_t n_cand, hipStream_t s) {
  if (n_cand == 0) return hipSuccess;
  hipLaunchKernelGGL(da_visit_kernel, dim3((unsigned)((n_cand + 255) / 256)), dim3(256), 0, s, a, n_cand);
  return hipGetLastError();
}

hipError_t launch_da_accept(const DaArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(da_accept_kernel, dim3((unsigned)a.M), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace dfit
