// Differential evolution over log10(tau), DE/rand/1/bin (Storn & Price 1997;
// the paper's DE-DLS alternative, Sec. III-A), one population per material,
// generation-synchronous: all trials of generation t are built from the
// population as it stood before it, evaluated in one batched cost launch,
// and each member is replaced by its trial when the trial's cost is not
// larger.  Random numbers: Philox4x64-10 with key (seed, material):
//   initial member p, coordinate d:   counter (d, p, 0, DE_INIT), word 0
//   trial of member i, generation t:  counter (i, t, 0, DE_TRIAL), words 0..2
//                                     the donors, word 3 the forced coordinate
//   coordinate d of that trial:       counter (i, t, d + 1, DE_CROSS), word 0
//                                     the crossover test, word 1 the redraw
//   scale factor of generation t:     counter (0, t, 0, DE_F), word 0
// Integers in [0, K) are ((w >> 32) * K) >> 32.  Every product and sum is
// rounded separately (no fused multiply-add), so a run is bit-reproducible.

#include <algorithm>

#include "common.hpp"
#include "rng.hpp"
#include "fit_eval.hpp"

namespace dfit {

namespace {

__device__ __forceinline__ int mat_of(const int64_t *off, int32_t M, int64_t c) {
  int lo = 0, hi = M - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int64_t below(uint64_t w, int64_t K) {
  return (int64_t)(((w >> 32) * (uint64_t)K) >> 32);
}

// k-th index of 0..P-1 that is not among the n sorted entries of `taken`
__device__ __forceinline__ int64_t skip(int64_t k, const int64_t *taken, int n) {
  for (int j = 0; j < n; ++j)
    if (k >= taken[j]) ++k;
  return k;
}

__device__ __forceinline__ void sort3(int64_t *v, int n) {
  for (int i = 1; i < n; ++i)
    for (int j = i; j > 0 && v[j] < v[j - 1]; --j) {
      const int64_t t = v[j];
      v[j] = v[j - 1];
      v[j - 1] = t;
    }
}

}  // namespace

__global__ __launch_bounds__(256) void de_init_kernel(const DeArgs a, int64_t n_cand) {
#pragma clang fp contract(off)
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < a.M) {
    a.best_cost[c] = INFINITY;
    a.best_idx[c] = -1;
  }
  if (c >= n_cand) return;
  const int m = mat_of(a.cand_off, a.M, c);
  const int64_t p = c - a.cand_off[m];
  const int N = a.n_poles[m];
  const double lo = a.lb[m], span = __dsub_rn(a.ub[m], a.lb[m]);
  for (int d = 0; d < N; ++d) {
    const U64x4 r = philox4x64((uint64_t)d, (uint64_t)p, 0, STREAM_DE_INIT, a.seed, (uint64_t)m);
    a.x[c * a.ld + d] = __dadd_rn(lo, __dmul_rn(span, unit53(r.w[0])));
  }
  a.fit[c] = INFINITY;
}

// one thread per member: its trial vector
__global__ __launch_bounds__(256) void de_trial_kernel(const DeArgs a, int64_t n_cand) {
#pragma clang fp contract(off)
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cand) return;
  const int32_t t = a.t_dev ? *a.t_dev : a.t;
  const int m = mat_of(a.cand_off, a.M, c);
  const int64_t c0 = a.cand_off[m];
  const int64_t P = a.cand_off[m + 1] - c0;
  const int64_t i = c - c0;
  const int N = a.n_poles[m];
  const int64_t ld = a.ld;
  const double *xi = a.x + c * ld;
  double *ui = a.u + c * ld;
  if (P < 4) {  // no three distinct donors: the trial is the target
    for (int d = 0; d < N; ++d) ui[d] = xi[d];
    return;
  }
  const uint64_t seed = a.seed, key1 = (uint64_t)m;
  const U64x4 fw = philox4x64(0, (uint64_t)t, 0, STREAM_DE_F, seed, key1);
  const double F = __dadd_rn(a.f_lo, __dmul_rn(__dsub_rn(a.f_hi, a.f_lo), unit53(fw.w[0])));
  const U64x4 w = philox4x64((uint64_t)i, (uint64_t)t, 0, STREAM_DE_TRIAL, seed, key1);
  int64_t taken[3] = {i, 0, 0};
  int64_t r1 = skip(below(w.w[0], P - 1), taken, 1);
  taken[1] = r1;
  sort3(taken, 2);
  int64_t r2 = skip(below(w.w[1], P - 2), taken, 2);
  taken[2] = r2;
  sort3(taken, 3);
  int64_t r3 = skip(below(w.w[2], P - 3), taken, 3);
  const int64_t jrand = below(w.w[3], N);
  const double *xa = a.x + (c0 + r1) * ld, *xb = a.x + (c0 + r2) * ld, *xc = a.x + (c0 + r3) * ld;
  const double lo = a.lb[m], hi = a.ub[m], span = __dsub_rn(hi, lo);
  for (int d = 0; d < N; ++d) {
    const U64x4 cr = philox4x64((uint64_t)i, (uint64_t)t, (uint64_t)d + 1, STREAM_DE_CROSS, seed, key1);
    double v = xi[d];
    if (unit53(cr.w[0]) < a.cr || d == jrand) {
      v = __dadd_rn(xa[d], __dmul_rn(F, __dsub_rn(xb[d], xc[d])));
      if (!(v >= lo && v <= hi)) v = __dadd_rn(lo, __dmul_rn(span, unit53(cr.w[1])));
    }
    ui[d] = v;
  }
}

// one block per material: greedy selection, then the lowest-index best
__global__ __launch_bounds__(256) void de_select_kernel(const DeArgs a) {
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
  for (int64_t p = tid; p < P; p += blockDim.x) {
    const int64_t c = c0 + p;
    const double f = a.cost_u[c];
    if (f <= a.fit[c]) {  // NaN never replaces
      a.fit[c] = f;
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

hipError_t launch_de_init(const DeArgs &a, int64_t n_cand, hipStream_t s) {
  const int64_t n = n_cand > a.M ? n_cand : a.M;
  hipLaunchKernelGGL(de_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, n_cand);
  return hipGetLastError();
}

hipError_t launch_de_trial(const DeArgs &a, int64_t n_cand, hipStream_t s) {
  if (n_cand == 0) return hipSuccess;
  hipLaunchKernelGGL(de_trial_kernel, dim3((unsigned)((n_cand + 255) / 256)), dim3(256), 0, s, a, n_cand);
  return hipGetLastError();
}

hipError_t launch_de_select(const DeArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(de_select_kernel, dim3((unsigned)a.M), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace dfit
