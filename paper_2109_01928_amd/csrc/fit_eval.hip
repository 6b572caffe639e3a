// Forward cost kernels of the Debye fitting library (the kernel itself is in
// fit_kernel.hpp; the adjoint instantiations are compiled in fit_grad.hip),
// the target-gradient kernel, and the dispatch by pole count.

#include "fit_kernel.hpp"

namespace dfit {

// --------------------------------------------------------------------------
// Target gradient: for each material and frequency point, the sum over its
// candidates (in index order) of gc * (2 r'_k) and gc * (2 r''_k + (I mu)_k),
// recomputed from the per-candidate records of the adjoint kernel (weights,
// mu, tau, eps_inf and the upstream gradient of each candidate).
// --------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void target_grad_kernel(const TargetGradArgs a, int32_t n_mats) {
  for (int32_t mi = blockIdx.y; mi < n_mats; mi += gridDim.y) {
  const int32_t m = a.mat_list[mi];
  const int64_t f0 = a.f_off[m], F = a.f_off[m + 1] - f0;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= F) continue;
  const double w = a.omega[f0 + k], er = a.eps_re[f0 + k], ei = a.eps_im[f0 + k];
  double sr = 0.0, si = 0.0;
  for (int64_t c = a.cand_off[m]; c < a.cand_off[m + 1]; ++c) {
    const double *rec = a.record + c * a.rec_ld;
    const double gc = rec[4 * N + 1];
    if (gc == 0.0) continue;
    double pr = 0.0, pi = 0.0, pm = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double x = w * rec[3 * N + i];
      const double R = rcp_nr(__builtin_fma(x, x, 1.0));
      const double I = x * R;
      pr = __builtin_fma(rec[i], R, pr);
      pi = __builtin_fma(rec[i], I, pi);
      pm = __builtin_fma(rec[2 * N + i], I, pm);
    }
    const double rr = (er - rec[4 * N]) - pr;
    const double ri = ei - pi;
    sr = __builtin_fma(gc, 2.0 * rr, sr);
    si = __builtin_fma(gc, __builtin_fma(2.0, ri, pm), si);
  }
  a.grad_re[f0 + k] = sr;
  a.grad_im[f0 + k] = si;
  }
}

// --------------------------------------------------------------------------
// dispatch tables
// --------------------------------------------------------------------------
template <int N> int lds_bytes_per_cand() { return Shape<N, pole_split_for(N)>::LDS_DOUBLES * 8; }

template <int N> hipError_t launch_target_n(const TargetGradArgs &a, int64_t max_f, int32_t n_mats, hipStream_t s) {
  dim3 grid((unsigned)((max_f + 255) / 256), (unsigned)(n_mats < 65535 ? n_mats : 65535));
  hipLaunchKernelGGL((target_grad_kernel<N>), grid, dim3(256), 0, s, a, n_mats);
  return hipGetLastError();
}

template <int... Ns> struct Table {
  static int pole_split(int n) {
    int r = 0;
    ((n == Ns ? (r = pole_split_for(Ns)) : 0), ...);
    return r;
  }
  static int lds(int n) {
    int r = 0;
    ((n == Ns ? (r = lds_bytes_per_cand<Ns>()) : 0), ...);
    return r;
  }
  static hipError_t fit(int n, const FitArgs &a, int64_t tiles, bool uni, hipStream_t s) {
    hipError_t e = hipErrorInvalidValue;
    ((n == Ns ? (e = launch_fit_variant<Ns, false>(a, tiles, uni, s)) : hipSuccess), ...);
    return e;
  }
  static hipError_t target(int n, const TargetGradArgs &a, int64_t max_f, int32_t n_mats, hipStream_t s) {
    hipError_t e = hipErrorInvalidValue;
    ((n == Ns ? (e = launch_target_n<Ns>(a, max_f, n_mats, s)) : hipSuccess), ...);
    return e;
  }
};
using AllN = Table<1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24>;

int pole_split(int n) { return AllN::pole_split(n); }
int lds_bytes_per_candidate(int n) { return AllN::lds(n); }
hipError_t launch_fit(int n, const FitArgs &a, int64_t n_tiles, bool grad, bool uni, hipStream_t s) {
  if (grad) return launch_fit_grad(n, a, n_tiles, uni, s);
  if (a.flags & FLAG_DD_REFINE) return launch_fit_dd(n, a, n_tiles, s);
  return AllN::fit(n, a, n_tiles, uni, s);
}
hipError_t launch_target_grad(int n, const TargetGradArgs &a, int64_t max_f, int32_t n_mats, hipStream_t s) {
  return AllN::target(n, a, max_f, n_mats, s);
}

}  // namespace dfit
