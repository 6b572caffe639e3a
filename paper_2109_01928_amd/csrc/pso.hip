// Particle swarm over log10(tau) (paper Sec. III-A/B: PSO determines the
// relaxation times; Kennedy & Eberhart 1995), one swarm per material, FP64.
// Random numbers: Philox4x64-10 with key (seed, material) and counter
// (dimension, particle, iteration, stream).  Every product and sum of the
// velocity update is rounded separately (no fused multiply-add) and evaluated
// in a fixed order, so a swarm is bit-reproducible from its seed.

#include <algorithm>

#include "common.hpp"
#include "rng.hpp"
#include "fit_eval.hpp"

namespace dfit {

__device__ __forceinline__ int material_of(const int64_t *off, int32_t M, int64_t c) {
  int lo = 0, hi = M - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void pso_init_kernel(const PsoArgs a, int64_t n_cand) {
#pragma clang fp contract(off)
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < a.M) {
    a.gbest_cost[c] = INFINITY;
    a.gbest_idx[c] = -1;
  }
  if (c >= n_cand) return;
  const int m = material_of(a.cand_off, a.M, c);
  const int64_t p = c - a.cand_off[m];
  const int N = a.n_poles[m];
  const double lo = a.lb[m], span = __dsub_rn(a.ub[m], a.lb[m]);
  for (int d = 0; d < N; ++d) {
    const U64x4 r = philox4x64((uint64_t)d, (uint64_t)p, 0, STREAM_PSO_INIT, a.seed, (uint64_t)m);
    const double x = __dadd_rn(lo, __dmul_rn(span, unit53(r.w[0])));
    const double v = __dmul_rn(span, __dsub_rn(__dmul_rn(2.0, unit53(r.w[1])), 1.0));
    a.x[c * a.ld + d] = x;
    a.v[c * a.ld + d] = v;
    a.pbest_x[c * a.ld + d] = x;
  }
  a.pbest_cost[c] = INFINITY;
}

hipError_t launch_pso_init(const PsoArgs &a, int64_t n_cand, hipStream_t s) {
  const int64_t n = n_cand > a.M ? n_cand : a.M;
  hipLaunchKernelGGL(pso_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, n_cand);
  return hipGetLastError();
}

// one block per material
__global__ __launch_bounds__(256) void pso_step_kernel(const PsoArgs a) {
#pragma clang fp contract(off)
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

  // personal bests (strict improvement; NaN never compares less)
  for (int64_t p = tid; p < P; p += blockDim.x) {
    const int64_t c = c0 + p;
    const double f = a.cost[c];
    if (f < a.pbest_cost[c]) {
      a.pbest_cost[c] = f;
      for (int d = 0; d < N; ++d) a.pbest_x[c * ld + d] = a.x[c * ld + d];
    }
  }
  __syncthreads();

  // lowest-index minimum of the personal bests
  double bv = INFINITY;
  int64_t bi = -1;
  for (int64_t p = tid; p < P; p += blockDim.x) {
    const double f = a.pbest_cost[c0 + p];
    if (bi < 0 || f < bv) {
      bv = f;
      bi = p;
    }
  }
  s_val[tid] = bv;
  s_idx[tid] = bi;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w) {
      const double v2 = s_val[tid + w];
      const int64_t i2 = s_idx[tid + w];
      const double v1 = s_val[tid];
      const int64_t i1 = s_idx[tid];
      const bool take = i2 >= 0 && (i1 < 0 || v2 < v1 || (v2 == v1 && i2 < i1));
      if (take) {
        s_val[tid] = v2;
        s_idx[tid] = i2;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int64_t best = s_idx[0];
    const int take = (best >= 0 && s_val[0] < a.gbest_cost[m]) ? 1 : 0;
    s_take = take;
    if (take) {
      a.gbest_cost[m] = s_val[0];
      a.gbest_idx[m] = best;
    }
    if (a.history) a.history[(int64_t)m * a.hist_ld + (t - 1)] = a.gbest_cost[m];
  }
  __syncthreads();
  if (s_take) {
    const int64_t best = s_idx[0];
    for (int d = tid; d < N; d += blockDim.x) a.gbest_x[(int64_t)m * ld + d] = a.pbest_x[(c0 + best) * ld + d];
  }
  if (!a.move) return;
  __syncthreads();

  const bool social = a.gbest_idx[m] >= 0;
  const double lo = a.lb[m], hi = a.ub[m];
  // one element (particle, dimension) per thread; the index split in 32-bit
  // arithmetic when the material's elements fit (always, at practical sizes)
  const bool idx32 = P * N < ((int64_t)1 << 31);
  for (int64_t e = tid; e < P * N; e += blockDim.x) {
    int64_t p;
    int d;
    if (idx32) {
      const uint32_t q = (uint32_t)e / (uint32_t)N;
      p = q;
      d = (int)((uint32_t)e - q * (uint32_t)N);
    } else {
      p = e / N;
      d = (int)(e - p * N);
    }
    const int64_t c = c0 + p;
    const U64x4 r = philox4x64((uint64_t)d, (uint64_t)p, (uint64_t)t, STREAM_PSO_STEP, a.seed, (uint64_t)m);
    const double r1 = unit53(r.w[0]), r2 = unit53(r.w[1]);
    const double xi = a.x[c * ld + d];
    double vel = __dmul_rn(a.inertia, a.v[c * ld + d]);
    vel = __dadd_rn(vel, __dmul_rn(__dmul_rn(a.c1, r1), __dsub_rn(a.pbest_x[c * ld + d], xi)));
    if (social) vel = __dadd_rn(vel, __dmul_rn(__dmul_rn(a.c2, r2), __dsub_rn(a.gbest_x[(int64_t)m * ld + d], xi)));
    a.v[c * ld + d] = vel;
    double xn = __dadd_rn(xi, vel);
    xn = xn < lo ? lo : (xn > hi ? hi : xn);
    a.x[c * ld + d] = xn;
  }
}

hipError_t launch_pso_step(const PsoArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(pso_step_kernel, dim3((unsigned)a.M), dim3(256), 0, s, a);
  return hipGetLastError();
}

// iteration counter of a replayed swarm graph (a kernel, so that graphs hold
// no memset nodes)
__global__ void set_counter_kernel(int32_t *c, int32_t v) { *c = v; }
__global__ void tick_kernel(int32_t *c) { *c = *c + 1; }

hipError_t launch_set_counter(int32_t *c, int32_t value, hipStream_t s) {
  hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(1), 0, s, c, value);
  return hipGetLastError();
}
__global__ __launch_bounds__(256) void fill_kernel(double *p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_tick(int32_t *c, hipStream_t s) {
  hipLaunchKernelGGL(tick_kernel, dim3(1), dim3(1), 0, s, c);
  return hipGetLastError();
}

}  // namespace dfit
