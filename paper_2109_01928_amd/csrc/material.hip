// Target synthesis for the relaxation models of the paper (Sec. II-B):
// Debye (Eq. 3), Havriliak-Negami (Eq. 4) and its Cole-Cole / Cole-Davidson
// special cases, Jonscher (the constant-Q form eps_inf + chi (j w/w_p)^(n-1)),
// CRIM (Eq. 6 with a = 1/2, Debye water in a lossless matrix) and a tabulated
// sum of HN terms with multiplicative Gaussian noise.  eps = eps' - j eps''
// (Eq. 1).  One thread per frequency point; FP64; the complex powers are taken
// on the principal branch in polar form.

#include "common.hpp"
#include "rng.hpp"
#include "fit_eval.hpp"

namespace dfit {

struct Cx {
  double re, im;
};
__device__ __forceinline__ Cx cmul(Cx a, Cx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ Cx cscale(Cx a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ Cx cadd(Cx a, Cx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ Cx cpolar(double mag, double ang) {
  double s, c;
  sincos(ang, &s, &c);
  return {mag * c, mag * s};
}
__device__ __forceinline__ Cx cinv(Cx a) {
  const double d = a.re * a.re + a.im * a.im;
  return {a.re / d, -a.im / d};
}
// principal square root
__device__ __forceinline__ Cx csqrt_p(Cx a) {
  const double r = hypot(a.re, a.im);
  double t = sqrt(0.5 * (r + fabs(a.re)));
  if (t == 0.0) return {0.0, 0.0};
  if (a.re >= 0.0) return {t, a.im / (2.0 * t)};
  return {fabs(a.im) / (2.0 * t), copysign(t, a.im)};
}

// One HN term with its parameter derivatives.  y = w tau0 > 0:
//   (j y)^alpha = y^alpha e^{j pi alpha / 2},  B = 1 + (j y)^alpha = |B| e^{j phi},
//   term = d_eps B^-beta = d_eps |B|^-beta e^{-j beta phi}
struct HnOut {
  Cx val;      // d_eps * B^-beta
  Cx d[5];     // d/d(eps_inf, d_eps, tau0, alpha, beta)
};
__device__ HnOut hn_term(double w, double d_eps, double tau0, double alpha, double beta, bool want_jac) {
  HnOut o;
  const double y = w * tau0;
  const double ly = log(y);
  const double pa = exp(alpha * ly);                   // y^alpha
  const Cx p = cpolar(pa, 0.5 * M_PI * alpha);         // (j y)^alpha
  const Cx B = {1.0 + p.re, p.im};
  const double lB = log(hypot(B.re, B.im));
  const double phi = atan2(B.im, B.re);
  const Cx Bmb = cpolar(exp(-beta * lB), -beta * phi);  // B^-beta
  o.val = cscale(Bmb, d_eps);
  if (want_jac) {
    const Cx Bmb1 = cmul(Bmb, cinv(B));                 // B^(-beta-1)
    const Cx k = cscale(Bmb1, -beta * d_eps);            // -beta d_eps B^(-beta-1)
    o.d[0] = {1.0, 0.0};
    o.d[1] = Bmb;
    o.d[2] = cmul(k, cscale(p, alpha / tau0));            // dB/dtau0 = alpha p / tau0
    o.d[3] = cmul(k, cmul(p, Cx{ly, 0.5 * M_PI}));        // dB/dalpha = p log(j y)
    o.d[4] = cscale(cmul(Bmb, Cx{lB, phi}), -d_eps);      // -d_eps B^-beta log B
  }
  return o;
}

__global__ __launch_bounds__(256) void material_kernel(const MaterialArgs a) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.n_freq) return;
  // material owning frequency g: largest m with f_off[m] <= g
  int lo = 0, hi = a.M - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.f_off[mid] <= g) lo = mid; else hi = mid - 1;
  }
  const int m = lo;
  const int64_t k = g - a.f_off[m];
  const double *p = a.params + (int64_t)m * 16;
  const int kind = a.kind[m];
  const double w = a.omega[g];
  Cx eps = {0.0, 0.0};
  Cx jac[5];
  bool have_jac = false;
  const bool want = a.jac != nullptr;
  switch (kind) {
  case 0: case 1: case 2: case 3: {
    const double alpha = (kind == 0 || kind == 3) ? 1.0 : p[3];
    const double beta = (kind == 0 || kind == 2) ? 1.0 : p[4];
    HnOut t = hn_term(w, p[1], p[2], alpha, beta, want);
    eps = {p[0] + t.val.re, t.val.im};
    if (want) {
      for (int i = 0; i < 5; ++i) jac[i] = t.d[i];
      have_jac = true;
    }
    break;
  }
  case 4: {  // Jonscher: eps_inf + chi (j w / w_p)^(n-1)
    const double y = w / p[2];
    const double e = p[3] - 1.0;
    const Cx t = cpolar(p[1] * exp(e * log(y)), 0.5 * M_PI * e);
    eps = {p[0] + t.re, t.im};
    break;
  }
  case 5: {  // CRIM, a = 1/2: sqrt(eps) = f sqrt(eps_w) + (1 - f) sqrt(eps_m)
    const double x = w * p[2];
    const double den = 1.0 + x * x;
    const Cx ew = {p[0] + p[1] / den, -p[1] * x / den};
    const Cx sw = csqrt_p(ew);
    const double sm = sqrt(p[4]);
    const Cx root = {p[3] * sw.re + (1.0 - p[3]) * sm, p[3] * sw.im};
    eps = cmul(root, root);
    break;
  }
  case 6: {  // eps_inf + sum of HN terms, times (1 + noise * gaussian)
    const int nt = (int)p[1];
    eps = {p[0], 0.0};
    for (int t = 0; t < nt && t < 3; ++t) {
      HnOut h = hn_term(w, p[2 + 4 * t], p[3 + 4 * t], p[4 + 4 * t], p[5 + 4 * t], false);
      eps = cadd(eps, h.val);
    }
    break;
  }
  default:
    eps = {NAN, NAN};
  }
  double er = eps.re, ei = -eps.im;
  if (kind == 6 && p[14] != 0.0) {
    // Box-Muller on two Philox uniforms (counter (k, 0, 0, noise stream), key (seed, m))
    const U64x4 r = philox4x64((uint64_t)k, 0, 0, STREAM_NOISE, a.noise_seed, (uint64_t)m);
    const double u1 = unit53(r.w[0]), u2 = unit53(r.w[1]);
    const double rad = sqrt(-2.0 * log(1.0 - u1));
    double s, c;
    sincos(2.0 * M_PI * u2, &s, &c);
    er = er * (1.0 + p[14] * (rad * c));
    ei = ei * (1.0 + p[14] * (rad * s));
  }
  a.eps_re[g] = er;
  a.eps_im[g] = ei;
  if (want) {
    double *J = a.jac + g * 10;
    for (int i = 0; i < 5; ++i) {
      J[2 * i] = have_jac ? jac[i].re : NAN;
      J[2 * i + 1] = have_jac ? -jac[i].im : NAN;
    }
  }
}

hipError_t launch_material(const MaterialArgs &a, hipStream_t s) {
  const int64_t blocks = (a.n_freq + 255) / 256;
  hipLaunchKernelGGL(material_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Parameter gradient of HN-family targets: grad_params[m][q] =
//   sum_k J[k][q][0] g_re[k] + J[k][q][1] g_im[k]   (q = eps_inf, d_eps, tau0,
// alpha, beta), one block per material, fixed-order tree reduction.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void material_vjp_kernel(int32_t M, const int64_t *f_off, const double *jac,
                                                          const double *g_re, const double *g_im, double *gp) {
  __shared__ double red[5][256];
  const int tid = threadIdx.x;
  for (int64_t m = blockIdx.x; m < M; m += gridDim.x) {
    const int64_t a = f_off[m], b = f_off[m + 1];
    double acc[5] = {0, 0, 0, 0, 0};
    for (int64_t k = a + tid; k < b; k += blockDim.x) {
      const double *J = jac + k * 10;
      const double gr = g_re[k], gi = g_im[k];
#pragma unroll
      for (int q = 0; q < 5; ++q) acc[q] = __builtin_fma(J[2 * q], gr, __builtin_fma(J[2 * q + 1], gi, acc[q]));
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) red[q][tid] = acc[q];
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if (tid < w)
#pragma unroll
        for (int q = 0; q < 5; ++q) red[q][tid] += red[q][tid + w];
      __syncthreads();
    }
    if (tid < 16) gp[m * 16 + tid] = tid < 5 ? red[tid][0] : 0.0;
    __syncthreads();
  }
}

hipError_t launch_material_vjp(int32_t M, const int64_t *f_off, const double *jac, const double *g_re,
                               const double *g_im, double *gp, hipStream_t s) {
  const int blocks = M < 65536 ? M : 65536;
  hipLaunchKernelGGL(material_vjp_kernel, dim3((unsigned)blocks), dim3(256), 0, s, M, f_off, jac, g_re, g_im, gp);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Debye basis materialised for inspection: re/im [n_cand][N][F] (coalesced
// along F).
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void basis_kernel(const double *omega, int64_t F, const double *theta, int64_t ld,
                                                   int64_t n_cand, int32_t N, double *re, double *im) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = blockIdx.y;  // c * N + i
  if (k >= F) return;
  const int64_t c = row / N;
  const int i = (int)(row - c * N);
  const double tau = exp10(theta[c * ld + i]);
  const double x = omega[k] * tau;
  const double R = rcp_nr(__builtin_fma(x, x, 1.0));
  re[row * F + k] = R;
  im[row * F + k] = x * R;
}

hipError_t launch_basis(const double *omega, int64_t F, const double *theta, int64_t ld, int64_t n_cand, int32_t N,
                        double *re, double *im, hipStream_t s) {
  const int64_t rows = n_cand * N;
  int64_t done = 0;
  // grid.y is limited to 65535 rows per launch
  while (done < rows) {
    const int64_t chunk = rows - done < 65535 ? rows - done : 65535;
    const int64_t c0 = done / N;  // chunks start at candidate boundaries
    const int64_t chunk_c = (chunk / N) > 0 ? chunk / N : 1;
    const int64_t nc = (c0 + chunk_c > n_cand) ? n_cand - c0 : chunk_c;
    dim3 grid((unsigned)((F + 255) / 256), (unsigned)(nc * N));
    hipLaunchKernelGGL(basis_kernel, grid, dim3(256), 0, s, omega, F, theta + c0 * ld, ld, nc, N, re + c0 * N * F,
                       im + c0 * N * F);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    done = (c0 + nc) * N;
  }
  return hipSuccess;
}

}  // namespace dfit

namespace dfit {

// --------------------------------------------------------------------------
// Average fractional error of a fitted expansion (the paper's accuracy figure,
// Sec. IV): 100 (mean_k |eps'_k - model'_k| / |eps'_k| + mean_k |eps''_k -
// model''_k| / |eps''_k|), model = eps_inf + sum_i w_i / (1 + j w_k tau_i);
// points with eps'' = 0 are left out of the second mean.  One 64-lane block
// per candidate, lanes strided over the frequencies, fixed-order reduction.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(64) void afe_kernel(const AfeArgs a) {
  const int64_t c = blockIdx.x;
  const int lane = threadIdx.x;
  int lo = 0, hi = a.M - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.cand_off[mid] <= c) lo = mid; else hi = mid - 1;
  }
  const int m = lo;
  const int64_t f0 = a.f_off[m], F = a.f_off[m + 1] - f0;
  const int N = a.n_poles[m];
  double tau[DFIT_MAX_POLES], w[DFIT_MAX_POLES];
  for (int i = 0; i < N; ++i) {
    tau[i] = exp10(a.theta[c * a.ld + i]);
    w[i] = a.weights[c * a.ld + i];
  }
  const double einf = a.eps_inf[c];
  double sr = 0.0, si = 0.0, ni = 0.0;
  for (int64_t k = lane; k < F; k += 64) {
    const double om = a.omega[f0 + k], er = a.eps_re[f0 + k], ei = a.eps_im[f0 + k];
    double mr = einf, mi = 0.0;
    for (int i = 0; i < N; ++i) {
      const double x = om * tau[i];
      const double R = 1.0 / __builtin_fma(x, x, 1.0);
      mr = __builtin_fma(w[i], R, mr);
      mi = __builtin_fma(w[i], x * R, mi);
    }
    sr += fabs(er - mr) / fabs(er);
    if (ei != 0.0) {
      si += fabs(ei - mi) / fabs(ei);
      ni += 1.0;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_xor(sr, off, 64);
    si += __shfl_xor(si, off, 64);
    ni += __shfl_xor(ni, off, 64);
  }
  if (lane == 0) a.afe[c] = 100.0 * (sr / (double)F + (ni > 0.0 ? si / ni : 0.0));
}

hipError_t launch_afe(const AfeArgs &a, int64_t n_cand, hipStream_t s) {
  if (n_cand == 0) return hipSuccess;
  if (n_cand > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(afe_kernel, dim3((unsigned)n_cand), dim3(64), 0, s, a);
  return hipGetLastError();
}

// dst entry e <- the first dst_off[e+1] - dst_off[e] points of the spectra of
// source material src_mat[e] (which has at least that many); one block per entry
__global__ __launch_bounds__(256) void gather_spectra_kernel(const int64_t *src_off, const int32_t *src_mat,
                                                             const int64_t *dst_off, const double *s0,
                                                             const double *s1, const double *s2, double *d0,
                                                             double *d1, double *d2) {
  const int64_t e = blockIdx.x;
  const int32_t m = src_mat[e];
  const int64_t a = src_off[m], b = dst_off[e], F = dst_off[e + 1] - b;
  for (int64_t k = threadIdx.x; k < F; k += blockDim.x) {
    d0[b + k] = s0[a + k];
    d1[b + k] = s1[a + k];
    d2[b + k] = s2[a + k];
  }
}

hipError_t launch_gather_spectra(int64_t n_entries, const int64_t *src_off, const int32_t *src_mat,
                                 const int64_t *dst_off, const double *s0, const double *s1, const double *s2,
                                 double *d0, double *d1, double *d2, hipStream_t s) {
  if (n_entries == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_spectra_kernel, dim3((unsigned)n_entries), dim3(256), 0, s, src_off, src_mat, dst_off, s0,
                     s1, s2, d0, d1, d2);
  return hipGetLastError();
}

// rows: dst[dst_row[e] * dst_ld + i] = src[src_row[e] * src_ld + i], i < n[e]
__global__ __launch_bounds__(64) void scatter_rows_kernel(int64_t n_entries, const int64_t *src_row,
                                                          const int64_t *dst_row, const int32_t *n,
                                                          const double *src, int64_t src_ld, double *dst,
                                                          int64_t dst_ld) {
  const int64_t e = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (e >= n_entries) return;
  for (int i = 0; i < n[e]; ++i) dst[dst_row[e] * dst_ld + i] = src[src_row[e] * src_ld + i];
}

hipError_t launch_scatter_rows(int64_t n_entries, const int64_t *src_row, const int64_t *dst_row, const int32_t *n,
                               const double *src, int64_t src_ld, double *dst, int64_t dst_ld, hipStream_t s) {
  if (n_entries == 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_rows_kernel, dim3((unsigned)((n_entries + 63) / 64)), dim3(64), 0, s, n_entries, src_row,
                     dst_row, n, src, src_ld, dst, dst_ld);
  return hipGetLastError();
}

}  // namespace dfit
