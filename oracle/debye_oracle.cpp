// Plain CPU reference ("oracle") for the multi-pole Debye fitting method of
// Majchrowska, Giannakis, Warren and Giannopoulos, "Modelling Arbitrary Complex
// Dielectric Properties - an automated implementation for gprMax" (2021).
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
// that the GPU library is checked against.  Only the test suite, the smoke
// check and the benchmark's CPU-baseline leg load it.  It shares no code,
// headers, tables or helpers with the GPU library.
//
// Everything is written from the definitions, in the order the paper states
// them, with no blocking, fusion or reordering:
//   * material models          Eq. (3) Debye, Eq. (4) Havriliak-Negami (and its
//                              Cole-Cole / Cole-Davidson special cases),
//                              Eq. (5) Jonscher, Eq. (6) CRIM, and a tabulated
//                              sum of HN terms with multiplicative noise
//                              (stand-in for user data, Sec. III-A)
//   * multi-Debye basis        Eq. (7) with the sign convention of Eq. (1)
//   * DLS weights              damped least squares on the loss part (Sec. III-A,
//                              Sec. III-B), solved by Householder QR of the
//                              stacked damped system (textbook LS)
//   * sign flip                negative weights flipped (Sec. III-B)
//   * eps_inf and cost         eps_inf = mean real-part misfit; cost = sum of
//                              squared real and imaginary residuals (Sec. III-B)
//   * adjoint gradient         variable-projection derivative of the cost
//   * complex-step gradient    the same forward map on complex numbers
//   * Philox4x64-10            Salmon et al., SC'11 (counter-based RNG)
//   * PSO                      Kennedy-Eberhart particle swarm (Sec. III-A)
//   * L-BFGS polish            Liu-Nocedal two-loop recursion, Armijo backtracking
//
// Floating point: FP64 (the paper's NumPy/SciPy implementation is FP64), built
// with -O2 -ffp-contract=off and no fast-math.  The forward model is templated
// on its scalar type: double is the contract, long double (x87 80-bit) is used
// to attribute disagreements, std::complex<double> gives complex-step
// derivatives.
//
// Parity pins for every function live in tests/test_oracle_*.py.

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include <quadmath.h>

#ifdef _OPENMP
#include <omp.h>
#endif

// quad precision (binary128, libquadmath) for the third instance of the
// forward map: the reference that shows which of the FP64 and 80-bit results
// is off where they disagree.  The few elementary functions the forward map
// calls are given binary128 overloads.
using f128 = __float128;
namespace std {
inline f128 sqrt(f128 x) { return sqrtq(x); }
inline f128 fabs(f128 x) { return fabsq(x); }
}  // namespace std

namespace {

using cd = std::complex<double>;

// Status codes (shared meaning with the library's public header, defined here
// independently).
enum { ST_OK = 0, ST_BADINPUT = 1, ST_SINGULAR = 2 };
enum { FLAG_NO_SIGN_FLIP = 1u };

// Largest |log10 tau| accepted (relaxation times 1e-30 .. 1e30 s); beyond it
// a candidate is reported BADINPUT.
constexpr double THETA_LIMIT = 30.0;
constexpr double LN10 = 2.302585092994045684017991454684364208;

// ---------------------------------------------------------------------------
// scalar helpers so that one template serves double, long double and the
// complex-step type
// ---------------------------------------------------------------------------
inline double re(double x) { return x; }
inline long double re(long double x) { return x; }
inline f128 re(f128 x) { return x; }
inline double re(const cd &x) { return x.real(); }

// |z| written as z*sign(Re z): equal to fabs for real types and the analytic
// continuation needed by the complex-step method.
template <class T> inline T flip_abs(const T &z) { return re(z) < 0 ? T(-z) : z; }

template <class T> inline T pow10_t(const T &t) { return std::pow(T(10), t); }
inline double pow10_t(const double &t) { return std::pow(10.0, t); }
inline long double pow10_t(const long double &t) { return std::pow(10.0L, t); }
inline f128 pow10_t(const f128 &t) { return powq(10, t); }

template <class T> inline bool finite_t(const T &x) { return std::isfinite(re(x)); }
inline bool finite_t(const cd &x) { return std::isfinite(x.real()) && std::isfinite(x.imag()); }
inline bool finite_t(const f128 &x) { return finiteq(x) != 0; }

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11).  Counter c[4], key k[2].
// ---------------------------------------------------------------------------
inline void mulhilo64(uint64_t a, uint64_t b, uint64_t &hi, uint64_t &lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  hi = (uint64_t)(p >> 64);
  lo = (uint64_t)p;
}

void philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c0, hi0, lo0);
    mulhilo64(M1, c2, hi1, lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    uint64_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// uniform double in [0, 1) from the top 53 bits of a 64-bit word
inline double u01(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

// Stream identifiers used as the last counter word.
enum { STREAM_PSO_INIT = 0, STREAM_PSO_STEP = 1, STREAM_NOISE = 2, STREAM_DE_INIT = 3, STREAM_DE_TRIAL = 4,
       STREAM_DE_CROSS = 5, STREAM_DE_F = 6, STREAM_DA_INIT = 7, STREAM_DA_VISIT = 8, STREAM_DA_ACCEPT = 9 };

// ---------------------------------------------------------------------------
// Material models (relaxation functions).  eps = eps' - j eps'' (Eq. 1).
// ---------------------------------------------------------------------------
enum {
  KIND_DEBYE = 0,    // Eq. 3:  (eps_inf, d_eps, tau0)
  KIND_HN = 1,       // Eq. 4:  (eps_inf, d_eps, tau0, alpha, beta)
  KIND_CC = 2,       // Eq. 4 with beta = 1
  KIND_CD = 3,       // Eq. 4 with alpha = 1
  KIND_JONSCHER = 4, // (eps_inf, chi, omega_p, n): eps_inf + chi (j w/w_p)^(n-1)
  KIND_CRIM = 5,     // Eq. 6, a = 1/2, water Debye phase + lossless matrix:
                     // (eps_inf_w, d_eps_w, tau_w, f_w, eps_m)
  KIND_HNSUM = 6,    // (eps_inf, n_terms, [d_eps, tau0, alpha, beta] x 3, noise)
  N_KINDS = 7
};
constexpr int PARAM_STRIDE = 16;

// One Havriliak-Negami term d_eps / (1 + (j w tau0)^alpha)^beta, principal
// branches, written with complex library arithmetic (Eq. 4).
inline cd hn_term(double w, double d_eps, double tau0, double alpha, double beta) {
  cd jwt(0.0, w * tau0);
  cd p = std::pow(jwt, alpha);
  cd base = 1.0 + p;
  return d_eps / std::pow(base, beta);
}

// d eps / d(eps_inf, d_eps, tau0, alpha, beta) for one HN term (+eps_inf).
inline void hn_term_jac(double w, double d_eps, double tau0, double alpha, double beta, cd out[5]) {
  cd jwt(0.0, w * tau0);
  cd p = std::pow(jwt, alpha);
  cd base = 1.0 + p;
  cd bmb = std::pow(base, -beta);                 // base^-beta
  cd bmb1 = std::pow(base, -beta - 1.0);          // base^(-beta-1)
  out[0] = cd(1.0, 0.0);
  out[1] = bmb;
  out[2] = -beta * d_eps * bmb1 * (alpha * p / tau0);
  out[3] = -beta * d_eps * bmb1 * (p * std::log(jwt));
  out[4] = -d_eps * bmb * std::log(base);
}

int material_one(int kind, const double *p, int64_t F, const double *omega, uint64_t noise_seed,
                 int64_t mat_index, double *eps_re, double *eps_im, double *jac) {
  if (kind < 0 || kind >= N_KINDS) return -1;
  for (int64_t k = 0; k < F; ++k) {
    const double w = omega[k];
    cd eps;
    switch (kind) {
    case KIND_DEBYE:
      eps = p[0] + p[1] / cd(1.0, w * p[2]);
      break;
    case KIND_HN:
      eps = p[0] + hn_term(w, p[1], p[2], p[3], p[4]);
      break;
    case KIND_CC:
      eps = p[0] + hn_term(w, p[1], p[2], p[3], 1.0);
      break;
    case KIND_CD:
      eps = p[0] + hn_term(w, p[1], p[2], 1.0, p[4]);
      break;
    case KIND_JONSCHER: {
      cd jy(0.0, w / p[2]);
      eps = p[0] + p[1] * std::pow(jy, p[3] - 1.0);
      break;
    }
    case KIND_CRIM: {
      cd eps_w = p[0] + p[1] / cd(1.0, w * p[2]);
      cd root = p[3] * std::sqrt(eps_w) + (1.0 - p[3]) * std::sqrt(cd(p[4], 0.0));
      eps = root * root;
      break;
    }
    case KIND_HNSUM: {
      int nt = (int)p[1];
      eps = cd(p[0], 0.0);
      for (int t = 0; t < nt && t < 3; ++t)
        eps += hn_term(w, p[2 + 4 * t], p[3 + 4 * t], p[4 + 4 * t], p[5 + 4 * t]);
      break;
    }
    }
    double er = eps.real(), ei = -eps.imag();
    if (kind == KIND_HNSUM && p[14] != 0.0) {
      // multiplicative Gaussian noise, Box-Muller on Philox uniforms
      uint64_t ctr[4] = {(uint64_t)k, 0, 0, STREAM_NOISE};
      uint64_t key[2] = {noise_seed, (uint64_t)mat_index};
      uint64_t r[4];
      philox4x64_10(ctr, key, r);
      double u1 = u01(r[0]), u2 = u01(r[1]);
      double rad = std::sqrt(-2.0 * std::log(1.0 - u1));
      double n1 = rad * std::cos(2.0 * M_PI * u2);
      double n2 = rad * std::sin(2.0 * M_PI * u2);
      er = er * (1.0 + p[14] * n1);
      ei = ei * (1.0 + p[14] * n2);
    }
    eps_re[k] = er;
    eps_im[k] = ei;
    if (jac) {
      double *J = jac + k * 10;
      if (kind <= KIND_CD) {
        double a = (kind == KIND_CD || kind == KIND_DEBYE) ? 1.0 : p[3];
        double b = (kind == KIND_CC || kind == KIND_DEBYE) ? 1.0 : p[4];
        cd d[5];
        hn_term_jac(w, p[1], p[2], a, b, d);
        for (int q = 0; q < 5; ++q) {
          J[2 * q] = d[q].real();
          J[2 * q + 1] = -d[q].imag();
        }
      } else {
        for (int q = 0; q < 10; ++q) J[q] = std::numeric_limits<double>::quiet_NaN();
      }
    }
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Multi-Debye basis, Eq. (7) split by Eq. (1):
//   1/(1 + j w tau) = R - j I,  R = 1/(1+x^2),  I = x/(1+x^2),  x = w tau
// ---------------------------------------------------------------------------
template <class T> inline void basis_point(double w, const T &tau, T &R, T &I) {
  T x = w * tau;
  T den = T(1) + x * x;
  R = T(1) / den;
  I = x / den;
}

// ---------------------------------------------------------------------------
// Forward map for one candidate.
// ---------------------------------------------------------------------------
template <class T> struct Fit {
  int status = ST_OK;
  T cost{}, eps_inf{};
  std::vector<T> tau, d, z, w;      // N
  std::vector<T> R, I;              // [F][N]
  std::vector<T> rre, rim;          // residuals, F
  std::vector<T> Rqr;               // N x N upper factor of the scaled damped system
};

template <class T>
void fit_solve(Fit<T> &out, int64_t F, const T *eps_re, const T *eps_im, int N, double damping, unsigned flags);

template <class T>
Fit<T> fit_forward(int64_t F, const double *omega, const T *eps_re, const T *eps_im, int N,
                   const T *theta, double damping, unsigned flags) {
  Fit<T> out;
  const double nan = std::numeric_limits<double>::quiet_NaN();
  out.cost = T(nan);
  out.eps_inf = T(nan);
  out.z.assign(N, T(nan));
  out.w.assign(N, T(nan));

  // input checks: non-finite data, or |log10 tau| beyond the accepted range
  bool bad = false;
  for (int i = 0; i < N; ++i)
    if (!finite_t(theta[i]) || std::fabs(re(theta[i])) > THETA_LIMIT) bad = true;
  for (int64_t k = 0; k < F; ++k)
    if (!std::isfinite(omega[k]) || !finite_t(eps_re[k]) || !finite_t(eps_im[k])) bad = true;
  if (bad) { out.status = ST_BADINPUT; return out; }

  // step 1: relaxation times and basis
  out.tau.resize(N);
  for (int i = 0; i < N; ++i) out.tau[i] = pow10_t(theta[i]);
  out.R.resize((size_t)F * N);
  out.I.resize((size_t)F * N);
  for (int64_t k = 0; k < F; ++k)
    for (int i = 0; i < N; ++i)
      basis_point(omega[k], out.tau[i], out.R[k * N + i], out.I[k * N + i]);
  fit_solve(out, F, eps_re, eps_im, N, damping, flags);
  return out;
}

// Steps 2-5 on the basis already held in out.R, out.I (row k, column i).
template <class T>
void fit_solve(Fit<T> &out, int64_t F, const T *eps_re, const T *eps_im, int N, double damping, unsigned flags) {
  // step 2: Marquardt scaling d_i = ||I_{:,i}||_2, then the damped least
  // squares  min || (I D^-1) zt - eps'' ||^2 + damping ||zt||^2  solved by
  // Householder QR of the stacked matrix [I D^-1 ; sqrt(damping) Id_N].
  out.d.resize(N);
  for (int i = 0; i < N; ++i) {
    T s = T(0);
    for (int64_t k = 0; k < F; ++k) s += out.I[k * N + i] * out.I[k * N + i];
    out.d[i] = std::sqrt(s);
    if (!(re(out.d[i]) > 0)) { out.status = ST_SINGULAR; out.cost = T(INFINITY); return; }
  }
  const int64_t m = F + N;
  std::vector<T> A((size_t)m * N, T(0)), y(m, T(0));
  for (int64_t k = 0; k < F; ++k) {
    for (int i = 0; i < N; ++i) A[k * N + i] = out.I[k * N + i] / out.d[i];
    y[k] = eps_im[k];
  }
  const T sq = std::sqrt(T(damping));
  for (int i = 0; i < N; ++i) A[(F + i) * N + i] = sq;

  for (int j = 0; j < N; ++j) {
    T sigma = T(0);
    for (int64_t r = j; r < m; ++r) sigma += A[r * N + j] * A[r * N + j];
    if (re(sigma) == 0) continue;
    T alpha = std::sqrt(sigma);
    if (re(A[j * N + j]) > 0) alpha = -alpha;
    // v = x - alpha e1 (stored in a scratch vector), H = Id - 2 v v^T / (v^T v)
    std::vector<T> v(m - j);
    for (int64_t r = j; r < m; ++r) v[r - j] = A[r * N + j];
    v[0] -= alpha;
    T vv = T(0);
    for (auto &e : v) vv += e * e;
    for (int c = j; c < N; ++c) {
      T dot = T(0);
      for (int64_t r = j; r < m; ++r) dot += v[r - j] * A[r * N + c];
      T f = T(2) * dot / vv;
      for (int64_t r = j; r < m; ++r) A[r * N + c] -= f * v[r - j];
    }
    T dot = T(0);
    for (int64_t r = j; r < m; ++r) dot += v[r - j] * y[r];
    T f = T(2) * dot / vv;
    for (int64_t r = j; r < m; ++r) y[r] -= f * v[r - j];
  }
  out.Rqr.assign((size_t)N * N, T(0));
  for (int i = 0; i < N; ++i)
    for (int j = i; j < N; ++j) out.Rqr[i * N + j] = A[i * N + j];

  // rank check, tolerance max(F, N) * unit roundoff * max|R_jj| (the usual
  // numerical-rank threshold); only reachable without damping
  {
    double rmax = 0, rmin = INFINITY;
    for (int i = 0; i < N; ++i) {
      double a = std::fabs((double)re(out.Rqr[i * N + i]));
      rmax = std::max(rmax, a);
      rmin = std::min(rmin, a);
    }
    if (rmin <= (double)std::max<int64_t>(F, N) * 0x1.0p-53 * rmax || rmax == 0) {
      out.status = ST_SINGULAR;
      out.cost = T(INFINITY);
      return;
    }
  }
  // back substitution  Rqr zt = (Q^T y)[0:N],  z = D^-1 zt
  std::vector<T> zt(N);
  for (int i = N - 1; i >= 0; --i) {
    T s = y[i];
    for (int j = i + 1; j < N; ++j) s -= out.Rqr[i * N + j] * zt[j];
    zt[i] = s / out.Rqr[i * N + i];
  }
  for (int i = 0; i < N; ++i) out.z[i] = zt[i] / out.d[i];

  // step 3: negative weights flipped (penalty reading of Sec. III-B)
  for (int i = 0; i < N; ++i) out.w[i] = (flags & FLAG_NO_SIGN_FLIP) ? out.z[i] : flip_abs(out.z[i]);

  // step 4: eps_inf = mean over frequencies of the real-part misfit
  T acc = T(0);
  for (int64_t k = 0; k < F; ++k) {
    T s = eps_re[k];
    for (int i = 0; i < N; ++i) s -= out.w[i] * out.R[k * N + i];
    acc += s;
  }
  out.eps_inf = acc / T((double)F);

  // step 5: residuals and cost (real + imaginary part)
  out.rre.resize(F);
  out.rim.resize(F);
  T cost = T(0);
  for (int64_t k = 0; k < F; ++k) {
    T a = eps_re[k] - out.eps_inf, b = eps_im[k];
    for (int i = 0; i < N; ++i) {
      a -= out.w[i] * out.R[k * N + i];
      b -= out.w[i] * out.I[k * N + i];
    }
    out.rre[k] = a;
    out.rim[k] = b;
    cost += a * a + b * b;
  }
  out.cost = cost;
}

// ---------------------------------------------------------------------------
// Variable-projection adjoint of the cost (derived for this method):
//   M z = I^T eps'',  M = I^T I + damping diag(I^T I)
//   g_w   = -2 (R^T r' + I^T r'')            (eps_inf is a mean: no term)
//   mu    = M^-1 (s o g_w),  s = sign(z) (or 1 without the flip)
//   dC/dtheta_i = -2 w_i (dR_i^T r' + dI_i^T r'') + mu_i dI_i^T (eps'' - I z)
//                 - z_i dI_i^T (I mu) - 2 damping mu_i z_i dI_i^T I_i
//   dC/deps'_k  = 2 r'_k,   dC/deps''_k = 2 r''_k + (I mu)_k
// with dR/dtheta = -2 ln10 x^2 R^2 and dI/dtheta = ln10 x R^2 (1 - x^2).
// M is applied through the QR factor: M = D Rqr^T Rqr D.
// ---------------------------------------------------------------------------
// g_w = -2 (R^T r' + I^T r'') and mu = D^-1 Rqr^-1 Rqr^-T D^-1 (s o g_w),
// the adjoint vector of the weights (M^-1 through the QR factor)
template <class T> std::vector<T> adjoint_mu(const Fit<T> &f, int64_t F, int N, unsigned flags) {
  std::vector<T> gw(N, T(0)), sg(N);
  for (int i = 0; i < N; ++i) {
    T s = T(0);
    for (int64_t k = 0; k < F; ++k) s += f.R[k * N + i] * f.rre[k] + f.I[k * N + i] * f.rim[k];
    gw[i] = T(-2) * s;
    sg[i] = (flags & FLAG_NO_SIGN_FLIP) ? T(1) : (f.z[i] < 0 ? T(-1) : T(1));
  }
  std::vector<T> u(N), v(N), mu(N);
  for (int i = 0; i < N; ++i) {
    T s = sg[i] * gw[i] / f.d[i];
    for (int j = 0; j < i; ++j) s -= f.Rqr[j * N + i] * u[j];
    u[i] = s / f.Rqr[i * N + i];
  }
  for (int i = N - 1; i >= 0; --i) {
    T s = u[i];
    for (int j = i + 1; j < N; ++j) s -= f.Rqr[i * N + j] * v[j];
    v[i] = s / f.Rqr[i * N + i];
  }
  for (int i = 0; i < N; ++i) mu[i] = v[i] / f.d[i];
  return mu;
}

struct GradOut {
  int status;
  double cost;
  std::vector<double> g_theta, g_re, g_im;
};

GradOut fit_grad(int64_t F, const double *omega, const double *eps_re, const double *eps_im, int N,
                 const double *theta, double damping, unsigned flags) {
  Fit<double> f = fit_forward<double>(F, omega, eps_re, eps_im, N, theta, damping, flags);
  GradOut g;
  g.status = f.status;
  g.cost = f.cost;
  const double nan = std::numeric_limits<double>::quiet_NaN();
  g.g_theta.assign(N, nan);
  g.g_re.assign(F, nan);
  g.g_im.assign(F, nan);
  if (f.status != ST_OK) return g;

  const std::vector<double> mu = adjoint_mu(f, F, N, flags);

  std::vector<double> Iz(F), Imu(F);
  for (int64_t k = 0; k < F; ++k) {
    double a = 0, b = 0;
    for (int i = 0; i < N; ++i) {
      a += f.I[k * N + i] * f.z[i];
      b += f.I[k * N + i] * mu[i];
    }
    Iz[k] = a;
    Imu[k] = b;
  }
  for (int i = 0; i < N; ++i) {
    double t1 = 0, t2 = 0, t3 = 0, t4 = 0;
    for (int64_t k = 0; k < F; ++k) {
      double x = omega[k] * f.tau[i];
      double R = f.R[k * N + i], I = f.I[k * N + i];
      double dR = -2.0 * LN10 * x * x * R * R;
      double dI = LN10 * x * R * R * (1.0 - x * x);
      t1 += dR * f.rre[k] + dI * f.rim[k];
      t2 += dI * (eps_im[k] - Iz[k]);
      t3 += dI * Imu[k];
      t4 += dI * I;
    }
    g.g_theta[i] = -2.0 * f.w[i] * t1 + mu[i] * t2 - f.z[i] * t3 - 2.0 * damping * mu[i] * f.z[i] * t4;
  }
  for (int64_t k = 0; k < F; ++k) {
    g.g_re[k] = 2.0 * f.rre[k];
    g.g_im[k] = 2.0 * f.rim[k] + Imu[k];
  }
  return g;
}

// ---------------------------------------------------------------------------
// Sensitivity of the cost to the rounding of the basis.  Any FP64 evaluation
// works with R and I rounded to a few units of roundoff u; to first order the
// cost then moves by up to  u * sum_ki (|dC/dR_ki R_ki| + |dC/dI_ki I_ki|),
// with the total derivatives (weights and eps_inf following the basis)
//   dC/dR_ki = -2 w_i r'_k         (eps_inf is a mean and sum_k r'_k = 0)
//   dC/dI_ki = -2 w_i r''_k + mu_i (eps'' - I z)_k - z_i (I mu)_k - 2 damping z_i mu_i I_ki,
// the same adjoint as the theta gradient before its contraction with dR/dtheta
// and dI/dtheta.  cond = that sum / C is the relative condition number of the
// cost under componentwise relative perturbations of the basis; computed in
// 80-bit arithmetic.  Returns the status; cond = NaN unless ST_OK.
// ---------------------------------------------------------------------------
int basis_sensitivity(int64_t F, const double *omega, const double *eps_re, const double *eps_im, int N,
                      const double *theta, double damping, unsigned flags, double *dCdR, double *dCdI,
                      double *cond) {
  using T = long double;
  std::vector<T> er(F), ei(F), th(N);
  for (int64_t k = 0; k < F; ++k) { er[k] = eps_re[k]; ei[k] = eps_im[k]; }
  for (int i = 0; i < N; ++i) th[i] = theta[i];
  Fit<T> f = fit_forward<T>(F, omega, er.data(), ei.data(), N, th.data(), damping, flags);
  *cond = std::numeric_limits<double>::quiet_NaN();
  if (f.status != ST_OK) return f.status;
  const std::vector<T> mu = adjoint_mu(f, F, N, flags);
  T sum = T(0);
  for (int64_t k = 0; k < F; ++k) {
    T iz = T(0), im = T(0);
    for (int i = 0; i < N; ++i) {
      iz += f.I[k * N + i] * f.z[i];
      im += f.I[k * N + i] * mu[i];
    }
    for (int i = 0; i < N; ++i) {
      const T dr = T(-2) * f.w[i] * f.rre[k];
      const T di = T(-2) * f.w[i] * f.rim[k] + mu[i] * (ei[k] - iz) - f.z[i] * im -
                   T(2) * T(damping) * f.z[i] * mu[i] * f.I[k * N + i];
      if (dCdR) dCdR[k * N + i] = (double)dr;
      if (dCdI) dCdI[k * N + i] = (double)di;
      sum += std::fabs(dr * f.R[k * N + i]) + std::fabs(di * f.I[k * N + i]);
    }
  }
  *cond = f.cost > 0 ? (double)(sum / f.cost) : INFINITY;
  return ST_OK;
}

// ---------------------------------------------------------------------------
// L-BFGS polish of one candidate (Liu & Nocedal 1989; two-loop recursion as in
// Nocedal & Wright, Algorithm 7.4), Armijo backtracking by halving.
// ---------------------------------------------------------------------------
struct LbfgsCfg {
  int steps, mem, max_trials;
  double c1;
};

// The inverse-Hessian product of L-BFGS, H v, by the two-loop recursion over
// the stored pairs (S[j], Y[j]), j = 0 oldest .. n-1 newest, rho_j = 1/(s_j.y_j),
// with the initial matrix gamma I, gamma = s.y / y.y of the newest pair (1
// without pairs): the first loop runs newest to oldest, the second oldest to
// newest (Nocedal & Wright, Algorithm 7.4 with the scaling of their eq. 7.20).
std::vector<double> lbfgs_two_loop(int N, const std::vector<std::vector<double>> &S,
                                   const std::vector<std::vector<double>> &Y, const std::vector<double> &rho,
                                   const std::vector<double> &v) {
  std::vector<double> q = v, a(S.size());
  for (int j = (int)S.size() - 1; j >= 0; --j) {
    double s = 0;
    for (int i = 0; i < N; ++i) s += S[j][i] * q[i];
    a[j] = rho[j] * s;
    for (int i = 0; i < N; ++i) q[i] -= a[j] * Y[j][i];
  }
  double gamma = 1.0;
  if (!S.empty()) {
    double sy = 0, yy = 0;
    for (int i = 0; i < N; ++i) { sy += S.back()[i] * Y.back()[i]; yy += Y.back()[i] * Y.back()[i]; }
    gamma = sy / yy;
  }
  for (int i = 0; i < N; ++i) q[i] *= gamma;
  for (int j = 0; j < (int)S.size(); ++j) {
    double s = 0;
    for (int i = 0; i < N; ++i) s += Y[j][i] * q[i];
    double b = rho[j] * s;
    for (int i = 0; i < N; ++i) q[i] += (a[j] - b) * S[j][i];
  }
  return q;
}

int lbfgs_one(int64_t F, const double *omega, const double *eps_re, const double *eps_im, int N,
              double *theta, double lb, double ub, double damping, unsigned flags, const LbfgsCfg &cfg,
              double *cost_hist, int32_t *rejected) {
  std::vector<double> th(theta, theta + N);
  GradOut g = fit_grad(F, omega, eps_re, eps_im, N, th.data(), damping, flags);
  double C = g.cost;
  std::vector<double> grad = g.g_theta;
  std::vector<std::vector<double>> S, Y;
  std::vector<double> rho;
  int taken = 0;
  for (int step = 0; step < cfg.steps; ++step) {
    if (cost_hist) cost_hist[step] = C;
    if (g.status != ST_OK || !std::isfinite(C)) continue;
    // search direction d = -H g
    const std::vector<double> q = lbfgs_two_loop(N, S, Y, rho, grad);
    std::vector<double> d(N);
    double gd = 0;
    for (int i = 0; i < N; ++i) { d[i] = -q[i]; gd += grad[i] * d[i]; }
    if (S.empty() || !(gd < 0)) {
      // steepest descent, scaled so the largest component moves one decade
      S.clear(); Y.clear(); rho.clear();
      double gmax = 0;
      for (int i = 0; i < N; ++i) gmax = std::max(gmax, std::fabs(grad[i]));
      if (!(gmax > 0)) continue;
      double sc = std::min(1.0, 1.0 / gmax);
      gd = 0;
      for (int i = 0; i < N; ++i) { d[i] = -grad[i] * sc; gd += grad[i] * d[i]; }
    }
    // Armijo backtracking alpha = 1, 1/2, 1/4, ... on the search box: the trial
    // point is projected onto [lb, ub] and the sufficient-decrease test uses the
    // projected displacement p:  C(trial) <= C + c1 min(g.p, 0)
    double alpha = 1.0;
    bool ok = false;
    std::vector<double> tt(N);
    double Ct = 0;
    for (int t = 0; t < cfg.max_trials; ++t) {
      double gp = 0;
      for (int i = 0; i < N; ++i) {
        double v = th[i] + alpha * d[i];
        tt[i] = v < lb ? lb : (v > ub ? ub : v);
        gp += grad[i] * (tt[i] - th[i]);
      }
      Fit<double> ft = fit_forward<double>(F, omega, eps_re, eps_im, N, tt.data(), damping, flags);
      Ct = ft.cost;
      // sufficient decrease along the projected step; where clamping makes
      // g.p positive, no increase at all (the polish never raises the cost)
      if (ft.status == ST_OK && Ct <= C + cfg.c1 * std::min(gp, 0.0)) { ok = true; break; }
      alpha *= 0.5;
    }
    if (!ok) continue;
    GradOut gt = fit_grad(F, omega, eps_re, eps_im, N, tt.data(), damping, flags);
    std::vector<double> s(N), y(N);
    double sy = 0;
    for (int i = 0; i < N; ++i) { s[i] = tt[i] - th[i]; y[i] = gt.g_theta[i] - grad[i]; sy += s[i] * y[i]; }
    if (sy > 1e-300) {
      S.push_back(s); Y.push_back(y); rho.push_back(1.0 / sy);
      if ((int)S.size() > cfg.mem) { S.erase(S.begin()); Y.erase(Y.begin()); rho.erase(rho.begin()); }
    } else if (rejected && (int)S.size() == cfg.mem) {
      ++*rejected;   // pair not stored while the history is full: its oldest pair stays live
    }
    th = tt;
    C = Ct;
    grad = gt.g_theta;
    g = gt;
    ++taken;
  }
  for (int i = 0; i < N; ++i) theta[i] = th[i];
  if (cost_hist) cost_hist[cfg.steps] = C;
  return taken;
}

int nthreads_or_default(int nthreads) {
#ifdef _OPENMP
  return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

inline int mat_of(const int64_t *cand_off, int32_t M, int64_t c) {
  // largest m with cand_off[m] <= c
  int lo = 0, hi = M - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) / 2;
    if (cand_off[mid] <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

} // namespace

// ===========================================================================
// C entry points (loaded with ctypes by the tests and the benchmark)
// ===========================================================================
extern "C" {

int orc_philox4x64_10(const uint64_t *ctr, const uint64_t *key, uint64_t *out) {
  philox4x64_10(ctr, key, out);
  return 0;
}

int orc_material_eval(int32_t M, const int8_t *kind, const double *params, const int64_t *f_off,
                      const double *omega, uint64_t noise_seed, double *eps_re, double *eps_im,
                      double *jac, int nthreads) {
  int bad = 0;
#pragma omp parallel for schedule(dynamic) num_threads(nthreads_or_default(nthreads)) reduction(| : bad)
  for (int32_t m = 0; m < M; ++m) {
    int64_t a = f_off[m], F = f_off[m + 1] - f_off[m];
    if (material_one(kind[m], params + (size_t)m * PARAM_STRIDE, F, omega + a, noise_seed, m,
                     eps_re + a, eps_im + a, jac ? jac + a * 10 : nullptr) != 0)
      bad |= 1;
  }
  return bad ? -1 : 0;
}

// as orc_material_eval, material m drawing its noise as material mat_index[m]
// of a larger batch (to evaluate a sample of that batch's materials)
int orc_material_eval_idx(int32_t M, const int8_t *kind, const double *params, const int64_t *f_off,
                          const double *omega, uint64_t noise_seed, const int64_t *mat_index, double *eps_re,
                          double *eps_im, int nthreads) {
  int bad = 0;
#pragma omp parallel for schedule(dynamic) num_threads(nthreads_or_default(nthreads)) reduction(| : bad)
  for (int32_t m = 0; m < M; ++m) {
    int64_t a = f_off[m], F = f_off[m + 1] - f_off[m];
    if (material_one(kind[m], params + (size_t)m * PARAM_STRIDE, F, omega + a, noise_seed, mat_index[m],
                     eps_re + a, eps_im + a, nullptr) != 0)
      bad |= 1;
  }
  return bad ? -1 : 0;
}

int orc_basis(const double *omega, int64_t F, const double *theta, int32_t N, double *re_out,
              double *im_out) {
  for (int i = 0; i < N; ++i) {
    double tau = pow10_t(theta[i]);
    for (int64_t k = 0; k < F; ++k) basis_point(omega[k], tau, re_out[i * F + k], im_out[i * F + k]);
  }
  return 0;
}

// Batched forward.  Candidate c of material m has log10 tau at theta[c*ld + i],
// i < n_poles[m]; weights use the same layout.  Any output pointer may be NULL.
int orc_fit_eval_batch(int32_t M, const int64_t *f_off, const int64_t *cand_off, const int32_t *n_poles,
                       const double *omega, const double *eps_re, const double *eps_im,
                       const double *theta, int64_t ld, double damping, uint32_t flags, double *cost,
                       double *weights, double *eps_inf, int8_t *status, int32_t precision,
                       int nthreads) {
  const int64_t P = cand_off[M];
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads_or_default(nthreads))
  for (int64_t c = 0; c < P; ++c) {
    int m = mat_of(cand_off, M, c);
    int64_t a = f_off[m], F = f_off[m + 1] - f_off[m];
    int N = n_poles[m];
    if (precision == 80 || precision == 128) {
      auto run = [&](auto zero) {
        using T = decltype(zero);
        std::vector<T> er(F), ei(F), th(N);
        for (int64_t k = 0; k < F; ++k) { er[k] = eps_re[a + k]; ei[k] = eps_im[a + k]; }
        for (int i = 0; i < N; ++i) th[i] = theta[c * ld + i];
        Fit<T> f = fit_forward<T>(F, omega + a, er.data(), ei.data(), N, th.data(), damping, flags);
        if (cost) cost[c] = (double)f.cost;
        if (eps_inf) eps_inf[c] = (double)f.eps_inf;
        if (status) status[c] = (int8_t)f.status;
        if (weights) for (int i = 0; i < N; ++i) weights[c * ld + i] = (double)f.w[i];
      };
      if (precision == 80) run((long double)0);
      else run((f128)0);
    } else {
      Fit<double> f = fit_forward<double>(F, omega + a, eps_re + a, eps_im + a, N, theta + c * ld, damping, flags);
      if (cost) cost[c] = f.cost;
      if (eps_inf) eps_inf[c] = f.eps_inf;
      if (status) status[c] = (int8_t)f.status;
      if (weights) for (int i = 0; i < N; ++i) weights[c * ld + i] = f.w[i];
    }
  }
  return 0;
}

// Batched adjoint.  grad_cost (NULL = ones) weights each candidate; the target
// gradients are summed over the candidates of each material (layout of omega).
int orc_fit_grad_batch(int32_t M, const int64_t *f_off, const int64_t *cand_off, const int32_t *n_poles,
                       const double *omega, const double *eps_re, const double *eps_im,
                       const double *theta, int64_t ld, double damping, uint32_t flags,
                       const double *grad_cost, double *cost, double *grad_theta, double *grad_re,
                       double *grad_im, int8_t *status, int nthreads) {
  const int64_t P = cand_off[M];
  std::vector<GradOut> all(P);
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads_or_default(nthreads))
  for (int64_t c = 0; c < P; ++c) {
    int m = mat_of(cand_off, M, c);
    int64_t a = f_off[m], F = f_off[m + 1] - f_off[m];
    int N = n_poles[m];
    all[c] = fit_grad(F, omega + a, eps_re + a, eps_im + a, N, theta + c * ld, damping, flags);
    double gc = grad_cost ? grad_cost[c] : 1.0;
    if (cost) cost[c] = all[c].cost;
    if (status) status[c] = (int8_t)all[c].status;
    if (grad_theta) for (int i = 0; i < N; ++i) grad_theta[c * ld + i] = gc * all[c].g_theta[i];
  }
  if (grad_re || grad_im) {
    for (int32_t m = 0; m < M; ++m) {
      int64_t a = f_off[m], F = f_off[m + 1] - f_off[m];
      for (int64_t k = 0; k < F; ++k) {
        double sr = 0, si = 0;
        for (int64_t c = cand_off[m]; c < cand_off[m + 1]; ++c) {
          double gc = grad_cost ? grad_cost[c] : 1.0;
          sr += gc * all[c].g_re[k];
          si += gc * all[c].g_im[k];
        }
        if (grad_re) grad_re[a + k] = sr;
        if (grad_im) grad_im[a + k] = si;
      }
    }
  }
  return 0;
}

// Complex-step derivative of the cost of one candidate: with respect to every
// log10 tau (grad_theta[N]) and every target value (grad_re/grad_im[F]).
int orc_fit_cs_grad(int64_t F, const double *omega, const double *eps_re, const double *eps_im, int32_t N,
                    const double *theta, double damping, uint32_t flags, double h, double *grad_theta,
                    double *grad_re, double *grad_im) {
  std::vector<cd> th(N), er(F), ei(F);
  for (int i = 0; i < N; ++i) th[i] = theta[i];
  for (int64_t k = 0; k < F; ++k) { er[k] = eps_re[k]; ei[k] = eps_im[k]; }
  if (grad_theta) {
    for (int i = 0; i < N; ++i) {
      th[i] = cd(theta[i], h);
      Fit<cd> f = fit_forward<cd>(F, omega, er.data(), ei.data(), N, th.data(), damping, flags);
      grad_theta[i] = f.cost.imag() / h;
      th[i] = theta[i];
    }
  }
  if (grad_re || grad_im) {
    for (int64_t k = 0; k < F; ++k) {
      if (grad_re) {
        er[k] = cd(eps_re[k], h);
        Fit<cd> f = fit_forward<cd>(F, omega, er.data(), ei.data(), N, th.data(), damping, flags);
        grad_re[k] = f.cost.imag() / h;
        er[k] = eps_re[k];
      }
      if (grad_im) {
        ei[k] = cd(eps_im[k], h);
        Fit<cd> f = fit_forward<cd>(F, omega, er.data(), ei.data(), N, th.data(), damping, flags);
        grad_im[k] = f.cost.imag() / h;
        ei[k] = eps_im[k];
      }
    }
  }
  return 0;
}

// Per-candidate internals for tests: unflipped LS solution z, scaling d and
// the residuals.  Returns the status.
// Cost from an explicitly given basis R, I ([F][N] row-major), steps 2-5 of
// the forward map; precision 64 or 80.
int orc_fit_from_basis(int64_t F, const double *R, const double *I, const double *eps_re, const double *eps_im,
                       int32_t N, double damping, uint32_t flags, int32_t precision, double *cost) {
  auto run = [&](auto tag) {
    using T = decltype(tag);
    Fit<T> f;
    f.R.assign(R, R + (size_t)F * N);
    f.I.assign(I, I + (size_t)F * N);
    std::vector<T> er(eps_re, eps_re + F), ei(eps_im, eps_im + F);
    f.cost = T(std::numeric_limits<double>::quiet_NaN());
    f.z.assign(N, T(0));
    f.w.assign(N, T(0));
    fit_solve(f, F, er.data(), ei.data(), N, damping, flags);
    *cost = (double)f.cost;
    return f.status;
  };
  return precision == 80 ? run((long double)0) : run(0.0);
}

int orc_fit_cond(int64_t F, const double *omega, const double *eps_re, const double *eps_im, int32_t N,
                 const double *theta, double damping, uint32_t flags, double *dCdR, double *dCdI, double *cond) {
  return basis_sensitivity(F, omega, eps_re, eps_im, N, theta, damping, flags, dCdR, dCdI, cond);
}

int orc_fit_cond_batch(int32_t M, const int64_t *f_off, const int64_t *cand_off, const int32_t *n_poles,
                       const double *omega, const double *eps_re, const double *eps_im, const double *theta,
                       int64_t ld, double damping, uint32_t flags, double *cond, int nthreads) {
  const int64_t P = cand_off[M];
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads_or_default(nthreads))
  for (int64_t c = 0; c < P; ++c) {
    int m = mat_of(cand_off, M, c);
    int64_t a = f_off[m], F = f_off[m + 1] - f_off[m];
    basis_sensitivity(F, omega + a, eps_re + a, eps_im + a, n_poles[m], theta + c * ld, damping, flags, nullptr,
                      nullptr, cond + c);
  }
  return 0;
}

int orc_fit_detail(int64_t F, const double *omega, const double *eps_re, const double *eps_im, int32_t N,
                   const double *theta, double damping, uint32_t flags, double *z, double *d,
                   double *rre, double *rim) {
  Fit<double> f = fit_forward<double>(F, omega, eps_re, eps_im, N, theta, damping, flags);
  if (f.status != ST_OK) return f.status;
  for (int i = 0; i < N; ++i) { if (z) z[i] = f.z[i]; if (d) d[i] = f.d[i]; }
  for (int64_t k = 0; k < F; ++k) { if (rre) rre[k] = f.rre[k]; if (rim) rim[k] = f.rim[k]; }
  return f.status;
}

// ---------------------------------------------------------------------------
// Particle swarm over log10 tau (one swarm per material).
//   init:  x = lb + (ub-lb) u0,  v = (ub-lb) (2 u1 - 1),  pbest_x = x,
//          best costs = +inf, no global best yet (gbest_idx = -1)
//          u0,u1 from Philox(key=(seed, m), ctr=(d, p, 0, STREAM_PSO_INIT)) words 0,1
//   step t (t >= 1) after the swarm has been evaluated (cost[c] = f(x_c)):
//     pbest: strict improvement; gbest: lowest-index argmin of pbest if strictly
//     better; history[m*hist_ld + t-1] = gbest cost;
//     move (if requested):  r1,r2 from Philox(key=(seed,m), ctr=(d,p,t,STREAM_PSO_STEP))
//       v = ((inertia*v) + ((c1*r1)*(pbest-x))) + ((c2*r2)*(gbest-x));  x = clamp(x+v)
// ---------------------------------------------------------------------------
int orc_pso_init(int32_t M, const int64_t *cand_off, const int32_t *n_poles, int64_t ld, const double *lb,
                 const double *ub, uint64_t seed, double *x, double *v, double *pbest_x,
                 double *pbest_cost, double *gbest_cost, int64_t *gbest_idx) {
  for (int32_t m = 0; m < M; ++m) {
    for (int64_t c = cand_off[m]; c < cand_off[m + 1]; ++c) {
      int64_t p = c - cand_off[m];
      for (int d = 0; d < n_poles[m]; ++d) {
        uint64_t ctr[4] = {(uint64_t)d, (uint64_t)p, 0, STREAM_PSO_INIT}, key[2] = {seed, (uint64_t)m}, r[4];
        philox4x64_10(ctr, key, r);
        double span = ub[m] - lb[m];
        x[c * ld + d] = lb[m] + span * u01(r[0]);
        v[c * ld + d] = span * (2.0 * u01(r[1]) - 1.0);
        pbest_x[c * ld + d] = x[c * ld + d];
      }
      pbest_cost[c] = INFINITY;
    }
    gbest_cost[m] = INFINITY;
    gbest_idx[m] = -1;
  }
  return 0;
}

int orc_pso_step(int32_t M, const int64_t *cand_off, const int32_t *n_poles, int64_t ld, const double *lb,
                 const double *ub, double inertia, double c1, double c2, uint64_t seed, int32_t t,
                 int32_t move, const double *cost, double *x, double *v, double *pbest_x,
                 double *pbest_cost, double *gbest_x, double *gbest_cost, int64_t *gbest_idx,
                 double *history, int64_t hist_ld) {
  for (int32_t m = 0; m < M; ++m) {
    const int N = n_poles[m];
    const int64_t c0 = cand_off[m], c1e = cand_off[m + 1];
    for (int64_t c = c0; c < c1e; ++c) {
      if (cost[c] < pbest_cost[c]) {
        pbest_cost[c] = cost[c];
        for (int d = 0; d < N; ++d) pbest_x[c * ld + d] = x[c * ld + d];
      }
    }
    // lowest-index argmin of the personal bests (NaN never wins)
    int64_t best = -1;
    for (int64_t c = c0; c < c1e; ++c) {
      if (std::isnan(pbest_cost[c])) continue;
      if (best < 0 || pbest_cost[c] < pbest_cost[best]) best = c;
    }
    if (best >= 0 && pbest_cost[best] < gbest_cost[m]) {
      gbest_cost[m] = pbest_cost[best];
      gbest_idx[m] = best - c0;
      for (int d = 0; d < N; ++d) gbest_x[m * ld + d] = pbest_x[best * ld + d];
    }
    if (history) history[m * hist_ld + (t - 1)] = gbest_cost[m];
    if (!move) continue;
    for (int64_t c = c0; c < c1e; ++c) {
      int64_t p = c - c0;
      for (int d = 0; d < N; ++d) {
        uint64_t ctr[4] = {(uint64_t)d, (uint64_t)p, (uint64_t)t, STREAM_PSO_STEP}, key[2] = {seed, (uint64_t)m}, r[4];
        philox4x64_10(ctr, key, r);
        double r1 = u01(r[0]), r2 = u01(r[1]);
        double xi = x[c * ld + d];
        double vel = inertia * v[c * ld + d];
        vel = vel + (c1 * r1) * (pbest_x[c * ld + d] - xi);
        // a swarm with no finite cost yet has no global best: no social term
        if (gbest_idx[m] >= 0) vel = vel + (c2 * r2) * (gbest_x[m * ld + d] - xi);
        v[c * ld + d] = vel;
        double xn = xi + vel;
        xn = xn < lb[m] ? lb[m] : (xn > ub[m] ? ub[m] : xn);
        x[c * ld + d] = xn;
      }
    }
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Differential evolution, DE/rand/1/bin (Storn & Price 1997), one population
// per material over log10 tau, generation-synchronous: every trial of a
// generation is built from the population as it stood at the start of it,
// all trials are evaluated together, then each member is replaced by its
// trial if the trial's cost is not larger.  Random numbers from Philox with
// key (seed, material):
//   initial member p, coordinate d:  ctr (d, p, 0, STREAM_DE_INIT), word 0
//   trial of member i, generation t: ctr (i, t, 0, STREAM_DE_TRIAL), words
//       0..2 -> the three donors, word 3 -> the coordinate always crossed
//   coordinate d of that trial:      ctr (i, t, d + 1, STREAM_DE_CROSS),
//       word 0 -> crossover test, word 1 -> redraw when out of the box
//   scale factor of generation t:    ctr (0, t, 0, STREAM_DE_F), word 0,
//       F = F_lo + (F_hi - F_lo) u  (dither per generation)
// An integer in [0, K) is ((w >> 32) * K) >> 32 (exact, no rounding).
// Donors r1, r2, r3 are distinct and differ from i: drawn from the remaining
// P-1, P-2, P-3 indices in increasing order.  A population of fewer than four
// members is not evolved (its trials are the targets).  A trial coordinate
// outside [lb, ub] is redrawn uniformly in the box.
// ---------------------------------------------------------------------------
inline int64_t draw_below(uint64_t w, int64_t K) { return (int64_t)(((w >> 32) * (uint64_t)K) >> 32); }

// the k-th (0-based) index of 0..P-1 that is not in `taken` (sorted, n entries)
inline int64_t skip_taken(int64_t k, const int64_t *taken, int n) {
  for (int j = 0; j < n; ++j)
    if (k >= taken[j]) ++k;
  return k;
}

void de_donors(uint64_t seed, int64_t m, int64_t i, int32_t t, int64_t P, int64_t r[3], uint64_t *jrand_w) {
  uint64_t ctr[4] = {(uint64_t)i, (uint64_t)t, 0, STREAM_DE_TRIAL}, key[2] = {seed, (uint64_t)m}, w[4];
  philox4x64_10(ctr, key, w);
  int64_t taken[3] = {i, 0, 0};
  r[0] = skip_taken(draw_below(w[0], P - 1), taken, 1);
  taken[1] = r[0];
  std::sort(taken, taken + 2);
  r[1] = skip_taken(draw_below(w[1], P - 2), taken, 2);
  taken[2] = r[1];
  std::sort(taken, taken + 3);
  r[2] = skip_taken(draw_below(w[2], P - 3), taken, 3);
  *jrand_w = w[3];
}

int orc_de_init(int32_t M, const int64_t *cand_off, const int32_t *n_poles, int64_t ld, const double *lb,
                const double *ub, uint64_t seed, double *x, double *fit, double *best_cost, int64_t *best_idx) {
  for (int32_t m = 0; m < M; ++m) {
    for (int64_t c = cand_off[m]; c < cand_off[m + 1]; ++c) {
      const int64_t p = c - cand_off[m];
      for (int d = 0; d < n_poles[m]; ++d) {
        uint64_t ctr[4] = {(uint64_t)d, (uint64_t)p, 0, STREAM_DE_INIT}, key[2] = {seed, (uint64_t)m}, w[4];
        philox4x64_10(ctr, key, w);
        x[c * ld + d] = lb[m] + (ub[m] - lb[m]) * u01(w[0]);
      }
      fit[c] = INFINITY;
    }
    best_cost[m] = INFINITY;
    best_idx[m] = -1;
  }
  return 0;
}

// trial vectors of generation t (t >= 1) from population x
int orc_de_trial(int32_t M, const int64_t *cand_off, const int32_t *n_poles, int64_t ld, const double *lb,
                 const double *ub, double f_lo, double f_hi, double cr, uint64_t seed, int32_t t, const double *x,
                 double *u) {
  for (int32_t m = 0; m < M; ++m) {
    const int64_t c0 = cand_off[m], P = cand_off[m + 1] - c0;
    const int N = n_poles[m];
    if (P == 0) continue;
    if (P < 4) {   // too few members for three distinct donors: the trial is the target
      for (int64_t c = c0; c < c0 + P; ++c)
        for (int d = 0; d < N; ++d) u[c * ld + d] = x[c * ld + d];
      continue;
    }
    uint64_t fctr[4] = {0, (uint64_t)t, 0, STREAM_DE_F}, key[2] = {seed, (uint64_t)m}, fw[4];
    philox4x64_10(fctr, key, fw);
    const double F = f_lo + (f_hi - f_lo) * u01(fw[0]);
    const double lo = lb[m], span = ub[m] - lb[m];
    for (int64_t i = 0; i < P; ++i) {
      int64_t r[3];
      uint64_t jw;
      de_donors(seed, m, i, t, P, r, &jw);
      const int64_t jrand = draw_below(jw, N);
      const double *xi = x + (c0 + i) * ld;
      const double *a = x + (c0 + r[0]) * ld, *b = x + (c0 + r[1]) * ld, *c = x + (c0 + r[2]) * ld;
      for (int d = 0; d < N; ++d) {
        uint64_t ctr[4] = {(uint64_t)i, (uint64_t)t, (uint64_t)d + 1, STREAM_DE_CROSS}, w[4];
        philox4x64_10(ctr, key, w);
        double v = xi[d];
        if (u01(w[0]) < cr || d == jrand) {
          const double diff = b[d] - c[d];
          const double step = F * diff;
          v = a[d] + step;
          if (!(v >= lo && v <= ub[m])) v = lo + span * u01(w[1]);
        }
        u[(c0 + i) * ld + d] = v;
      }
    }
  }
  return 0;
}

// greedy selection of generation t (t = 0: the initial population itself, u = x)
int orc_de_select(int32_t M, const int64_t *cand_off, const int32_t *n_poles, int64_t ld, int32_t t,
                  const double *u, const double *cost_u, double *x, double *fit, double *best_x, double *best_cost,
                  int64_t *best_idx, double *history, int64_t hist_ld) {
  for (int32_t m = 0; m < M; ++m) {
    const int64_t c0 = cand_off[m], c1 = cand_off[m + 1];
    const int N = n_poles[m];
    for (int64_t c = c0; c < c1; ++c)
      if (cost_u[c] <= fit[c]) {   // NaN never replaces
        fit[c] = cost_u[c];
        for (int d = 0; d < N; ++d) x[c * ld + d] = u[c * ld + d];
      }
    int64_t best = -1;
    for (int64_t c = c0; c < c1; ++c) {
      if (std::isnan(fit[c])) continue;
      if (best < 0 || fit[c] < fit[best]) best = c;
    }
    if (best >= 0 && fit[best] < best_cost[m]) {
      best_cost[m] = fit[best];
      best_idx[m] = best - c0;
      for (int d = 0; d < N; ++d) best_x[m * ld + d] = x[best * ld + d];
    }
    if (history) history[m * hist_ld + t] = best_cost[m];
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Exponential and logarithm written out from their textbook series, every
// operation rounded on its own, so that the annealing's random transforms are
// reproducible bit for bit by any IEEE double implementation of the same steps.
//   exp: x = k ln2 + r, k = rint(x / ln2), |r| <= ln2/2, ln2 split into a
//        20-bit head (k * head exact) and a tail (Cody & Waite 1980);
//        e^r = 1 + r (1 + r/2 (1 + r/3 (... (1 + r/17)))), then scaled by 2^k.
//   log: x = m 2^e, m in [sqrt(1/2), sqrt(2)); s = (m - 1)/(m + 1),
//        log m = 2 s (1 + s^2/3 + s^4/5 + ... + s^24/25) (the atanh series).
// ---------------------------------------------------------------------------
constexpr double LN2_HEAD = 0x1.62e42p-1, LN2_TAIL = 0x1.fdf473de6af28p-22;   // LN2_HEAD + LN2_TAIL = ln 2
constexpr double INV_LN2 = 0x1.71547652b82fep+0;

double series_exp(double x) {
  if (x != x) return x;
  if (x > 709.0) return INFINITY;
  if (x < -745.0) return 0.0;
  const double k = std::nearbyint(x * INV_LN2);
  const double r = (x - k * LN2_HEAD) - k * LN2_TAIL;
  double p = 1.0;
  for (int n = 17; n >= 1; --n) p = 1.0 + (r / (double)n) * p;
  return std::ldexp(p, (int)k);
}

double series_log(double x) {
  if (x != x || x < 0.0) return NAN;
  if (x == 0.0) return -INFINITY;
  if (x == INFINITY) return INFINITY;
  int e = 0;
  double m = std::frexp(x, &e);   // [1/2, 1)
  if (m < 0x1.6a09e667f3bcdp-1) {  // sqrt(1/2)
    m = 2.0 * m;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double q = 1.0 / 25.0;
  for (int k = 11; k >= 0; --k) q = q * z + 1.0 / (double)(2 * k + 1);
  const double lm = 2.0 * s * q;
  return (double)e * LN2_HEAD + ((double)e * LN2_TAIL + lm);
}

// ---------------------------------------------------------------------------
// Annealing (the paper's DA-DLS alternative, Sec. III-A): generalized
// simulated annealing (Tsallis & Stariolo 1996) as used by dual annealing,
// batched: the candidates of a material are independent Markov chains over
// log10 tau.  Generation t >= 1 (scalars from the series above):
//   visiting temperature  T(t) = T0 (2^(qv-1) - 1) / ((1 + t)^(qv-1) - 1)
//   acceptance temperature Ta(t) = T(t) / t
//   proposal  y_d = x_d + s(t) g_d, s(t) = T(t)^(1/(3-qv)) / sqrt(3 - qv),
//             g_d Student-t with nu = (3 - qv)/(qv - 1) degrees of freedom
//             (the one-dimensional visiting distribution), drawn by Bailey's
//             polar method, then wrapped into [lb, ub] periodically
//   accept    if f(y) < f(x); otherwise with probability
//             [1 - (1 - qa)(f(y) - f(x))/Ta]^(1/(1-qa)) when the bracket is
//             positive: u^(1-qa) < bracket
// Random numbers, Philox key (seed, material):
//   initial chain i, coordinate d:  ctr (d, i, 0, DA_INIT), word 0
//   proposal coordinate d:          ctr (d, i, t, DA_VISIT + 16 j), pairs of
//       words (0,1), (2,3) for the j-th round of the polar method (at most 16
//       rounds; g = 0 if none is accepted)
//   acceptance of chain i:          ctr (0, i, t, DA_ACCEPT), word 0
// ---------------------------------------------------------------------------
struct DaTemps { double visit_scale, accept_temp; };

DaTemps da_temps(double qv, double t0, int32_t t) {
  const double a = qv - 1.0;
  const double num = series_exp(a * series_log(2.0)) - 1.0;
  const double den = series_exp(a * series_log(1.0 + (double)t)) - 1.0;
  const double T = t0 * num / den;
  DaTemps r;
  r.visit_scale = series_exp(series_log(T) / (3.0 - qv)) / std::sqrt(3.0 - qv);
  r.accept_temp = T / (double)t;
  return r;
}

double student_t_polar(uint64_t seed, uint64_t m, uint64_t d, uint64_t i, uint64_t t, double nu) {
  for (int j = 0; j < 16; ++j) {
    uint64_t ctr[4] = {d, i, t, (uint64_t)(STREAM_DA_VISIT + 16 * j)}, key[2] = {seed, m}, w[4];
    philox4x64_10(ctr, key, w);
    for (int h = 0; h < 2; ++h) {
      const double u = 2.0 * u01(w[2 * h]) - 1.0, v = 2.0 * u01(w[2 * h + 1]) - 1.0;
      const double W = u * u + v * v;
      if (W > 0.0 && W <= 1.0) {
        double q = series_exp((-2.0 / nu) * series_log(W));
        if (q > 1e300) q = 1e300;
        return u * std::sqrt(nu * (q - 1.0) / W);
      }
    }
  }
  return 0.0;
}

// periodic wrap into [lo, hi]
inline double wrap_box(double y, double lo, double hi) {
  if (y >= lo && y <= hi) return y;
  const double span = hi - lo;
  double r = std::fmod(y - lo, span);
  if (r < 0.0) r = r + span;
  return lo + r;
}

int orc_series_exp_log(int64_t n, const double *x, double *ex, double *lg) {
  for (int64_t i = 0; i < n; ++i) {
    if (ex) ex[i] = series_exp(x[i]);
    if (lg) lg[i] = series_log(x[i]);
  }
  return 0;
}

int orc_student_t(uint64_t seed, int64_t n, double nu, double *out) {
  for (int64_t i = 0; i < n; ++i) out[i] = student_t_polar(seed, 0, 0, (uint64_t)i, 1, nu);
  return 0;
}

int orc_da_temps(double qv, double t0, int32_t t, double *visit_scale, double *accept_temp) {
  const DaTemps r = da_temps(qv, t0, t);
  *visit_scale = r.visit_scale;
  *accept_temp = r.accept_temp;
  return 0;
}

int orc_da_init(int32_t M, const int64_t *cand_off, const int32_t *n_poles, int64_t ld, const double *lb,
                const double *ub, uint64_t seed, double *x, double *fit, double *best_cost, int64_t *best_idx) {
  for (int32_t m = 0; m < M; ++m) {
    for (int64_t c = cand_off[m]; c < cand_off[m + 1]; ++c) {
      const int64_t i = c - cand_off[m];
      for (int d = 0; d < n_poles[m]; ++d) {
        uint64_t ctr[4] = {(uint64_t)d, (uint64_t)i, 0, STREAM_DA_INIT}, key[2] = {seed, (uint64_t)m}, w[4];
        philox4x64_10(ctr, key, w);
        x[c * ld + d] = lb[m] + (ub[m] - lb[m]) * u01(w[0]);
      }
      fit[c] = INFINITY;
    }
    best_cost[m] = INFINITY;
    best_idx[m] = -1;
  }
  return 0;
}

// proposals of generation t >= 1
int orc_da_visit(int32_t M, const int64_t *cand_off, const int32_t *n_poles, int64_t ld, const double *lb,
                 const double *ub, double qv, double t0, uint64_t seed, int32_t t, const double *x, double *y) {
  const DaTemps tp = da_temps(qv, t0, t);
  const double nu = (3.0 - qv) / (qv - 1.0);
  for (int32_t m = 0; m < M; ++m)
    for (int64_t c = cand_off[m]; c < cand_off[m + 1]; ++c) {
      const int64_t i = c - cand_off[m];
      for (int d = 0; d < n_poles[m]; ++d) {
        const double g = student_t_polar(seed, (uint64_t)m, (uint64_t)d, (uint64_t)i, (uint64_t)t, nu);
        y[c * ld + d] = wrap_box(x[c * ld + d] + tp.visit_scale * g, lb[m], ub[m]);
      }
    }
  return 0;
}

// acceptance of generation t (t = 0: the initial chains, all accepted)
int orc_da_accept(int32_t M, const int64_t *cand_off, const int32_t *n_poles, int64_t ld, double qv, double qa,
                  double t0, uint64_t seed, int32_t t, const double *y, const double *cost_y, double *x, double *fit,
                  double *best_x, double *best_cost, int64_t *best_idx, double *history, int64_t hist_ld) {
  const DaTemps tp = t > 0 ? da_temps(qv, t0, t) : DaTemps{0.0, 0.0};
  for (int32_t m = 0; m < M; ++m) {
    const int64_t c0 = cand_off[m], c1 = cand_off[m + 1];
    const int N = n_poles[m];
    for (int64_t c = c0; c < c1; ++c) {
      const double fy = cost_y[c], fx = fit[c];
      bool take;
      if (t == 0 || fy < fx) {
        take = !(fy != fy);
      } else if (fy != fy) {
        take = false;
      } else {
        const double z = 1.0 - (1.0 - qa) * (fy - fx) / tp.accept_temp;
        take = false;
        if (z > 0.0) {
          uint64_t ctr[4] = {0, (uint64_t)(c - c0), (uint64_t)t, STREAM_DA_ACCEPT}, key[2] = {seed, (uint64_t)m}, w[4];
          philox4x64_10(ctr, key, w);
          const double u = u01(w[0]);
          take = series_exp((1.0 - qa) * series_log(u)) < z;
        }
      }
      if (take) {
        fit[c] = fy;
        for (int d = 0; d < N; ++d) x[c * ld + d] = y[c * ld + d];
      }
    }
    // best visited state: the lowest-index minimum of the chains' accepted costs
    int64_t best = -1;
    for (int64_t c = c0; c < c1; ++c) {
      if (std::isnan(fit[c])) continue;
      if (best < 0 || fit[c] < fit[best]) best = c;
    }
    if (best >= 0 && fit[best] < best_cost[m]) {
      best_cost[m] = fit[best];
      best_idx[m] = best - c0;
      for (int d = 0; d < N; ++d) best_x[m * ld + d] = x[best * ld + d];
    }
    if (history) history[m * hist_ld + t] = best_cost[m];
  }
  return 0;
}

// L-BFGS polish of one candidate per material (theta[m*ld + i], in place),
// kept inside the search box [lb[m], ub[m]].  cost_hist (optional) receives
// steps+1 values per material.
int orc_lbfgs_batch(int32_t M, const int64_t *f_off, const int32_t *n_poles, const double *omega,
                    const double *eps_re, const double *eps_im, double *theta, int64_t ld, const double *lb,
                    const double *ub, double damping, uint32_t flags, int32_t steps, int32_t mem,
                    int32_t max_trials, double c1, double *cost_hist, int32_t *rejected, int nthreads) {
  LbfgsCfg cfg{steps, mem, max_trials, c1};
#pragma omp parallel for schedule(dynamic) num_threads(nthreads_or_default(nthreads))
  for (int32_t m = 0; m < M; ++m) {
    int64_t a = f_off[m], F = f_off[m + 1] - f_off[m];
    if (rejected) rejected[m] = 0;
    lbfgs_one(F, omega + a, eps_re + a, eps_im + a, n_poles[m], theta + m * ld, lb[m], ub[m], damping, flags, cfg,
              cost_hist ? cost_hist + (size_t)m * (steps + 1) : nullptr, rejected ? rejected + m : nullptr);
  }
  return 0;
}

// H v of the two-loop recursion for n stored pairs S, Y [n][N] (oldest
// first) with rho_j = 1 / (s_j . y_j).
int orc_lbfgs_two_loop(int32_t N, int32_t n, const double *S, const double *Y, const double *v, double *out) {
  std::vector<std::vector<double>> Sv(n), Yv(n);
  std::vector<double> rho(n);
  for (int j = 0; j < n; ++j) {
    Sv[j].assign(S + (size_t)j * N, S + (size_t)(j + 1) * N);
    Yv[j].assign(Y + (size_t)j * N, Y + (size_t)(j + 1) * N);
    double sy = 0;
    for (int i = 0; i < N; ++i) sy += Sv[j][i] * Yv[j][i];
    rho[j] = 1.0 / sy;
  }
  const std::vector<double> q = lbfgs_two_loop(N, Sv, Yv, rho, std::vector<double>(v, v + N));
  for (int i = 0; i < N; ++i) out[i] = q[i];
  return 0;
}

// Average fractional error (Sec. IV): mean |r'|/|eps'| + mean |r''|/|eps''|,
// in percent, for the model eps_inf + sum_n d_eps_n / (1 + j w tau_n).
// Frequencies with eps'' == 0 are left out of the imaginary mean.
double orc_afe(int64_t F, const double *omega, const double *eps_re, const double *eps_im, int32_t N,
               const double *d_eps, const double *tau, double eps_inf) {
  double sr = 0, si = 0;
  int64_t ni = 0;
  for (int64_t k = 0; k < F; ++k) {
    cd model(eps_inf, 0.0);
    for (int i = 0; i < N; ++i) model += d_eps[i] / cd(1.0, omega[k] * tau[i]);
    double mr = model.real(), mi = -model.imag();
    sr += std::fabs(eps_re[k] - mr) / std::fabs(eps_re[k]);
    if (eps_im[k] != 0) { si += std::fabs(eps_im[k] - mi) / std::fabs(eps_im[k]); ++ni; }
  }
  return 100.0 * (sr / (double)F + (ni ? si / (double)ni : 0.0));
}

int orc_num_threads(void) { return nthreads_or_default(0); }

} // extern "C"
