// Batched multi-Debye DLS cost evaluation and its variable-projection adjoint
// for gfx950 (MI355X), FP64.
//
// Method (paper Sec. III-B; Eq. 7 basis with the sign of Eq. 1):
//   tau_i = 10^theta_i, x_ki = w_k tau_i, R_ki = 1/(1+x^2), I_ki = x R_ki
//   weights: damped least squares on the loss part with Marquardt scaling,
//     (D^-1 G D^-1 + damping Id) zt = D^-1 b,  G = I^T I, b = I^T eps'', D = diag(G)^1/2,
//     z = D^-1 zt, solved by Cholesky plus one corrected-semi-normal-equations
//     step (a residual pass over the frequencies, I^T r accumulated with
//     compensation) because log-spaced Debye columns are nearly collinear;
//   flip: w = |z| (penalty for negative weights);
//   eps_inf = (sum_k eps'_k - sum_i w_i S_i) / F,  S_i = sum_k R_ki;
//   cost = sum_k (eps'_k - eps_inf - (R w)_k)^2 + (eps''_k - (I w)_k)^2.
//
// Work decomposition (one wavefront per work tile, one tile per 64-lane block):
//   - a candidate is served by SP x SF lanes: SP lanes split its poles (the
//     "ring" split below) and SF lanes split its frequency points;
//   - the 64/(SP*SF) candidates of a wave are listed by the plan (any mix of
//     materials with the same pole count);
//   - every F-reduction is a per-lane register accumulation followed by a
//     fixed butterfly over the SF lanes, so results are deterministic;
//   - passes: (1) Gram and right-hand side, (2) refinement residual (and,
//     for the adjoint, the column sums S), (3) cost; passes 1 and 2
//     recompute the basis in registers (it is never stored; four poles share
//     one reciprocal), pass 3 evaluates the model sums as rational functions
//     of w^2 (basis form as the fallback), and the adjoint adds pass 4.
//
// Ring split of the Gram matrix for SP > 1 poles-per-lane groups: the NP =
// NB*SP (padded) poles are placed on a ring; lane q owns poles q*NB .. q*NB+NB-1
// and accumulates, for each owned pole p and each offset d = 0..NP/2, the
// entry G(p, (p+d) mod NP).  Every unordered pair is covered (the d = NP/2
// entries twice, with bit-identical values), the work is balanced, and a lane
// only needs the basis values of the next NP/2 poles on the ring, which it
// receives from its neighbours by DPP quad permutes.  Padded poles get tau = 0,
// so their loss column is exactly zero and they drop out.

#pragma once

#include "common.hpp"
#include "fit_eval.hpp"

namespace dfit {

template <int N, int SP> struct Shape {
  static_assert(SP == 1 || SP == 2 || SP == 4, "pole split must be 1, 2 or 4");
  static constexpr int NB = (N + SP - 1) / SP;               // poles owned per lane
  static constexpr int NP = NB * SP;                         // padded ring size
  static constexpr int D = (SP == 1) ? 0 : NP / 2;           // ring half width
  static constexpr int NV = (SP == 1) ? N : NB + D;          // basis values seen by a lane
  static constexpr int NG = (SP == 1) ? N * (N + 1) / 2 : NB * (D + 1);  // Gram accumulators
  static constexpr int NT = N * (N + 1) / 2;                 // packed triangle
  // per candidate: the parked factor (SP == 1), or the whole solve (SP > 1)
  static constexpr int LDS_DOUBLES = (SP == 1) ? N * (N + 1) / 2 : N * (N + 1) / 2 + 5 * N;
};

constexpr __host__ __device__ int tri(int n, int i, int j) { return i * n - (i * (i - 1)) / 2 + (j - i); }

// value of block t (owned by lane (q + t) mod SP) of a lane's ring view
template <int SP> __device__ __forceinline__ double ring_fetch(double v, int t) {
  if constexpr (SP == 2) {
    return dpp_quad<QP_SWAP1>(v);
  } else {
    return t == 1 ? dpp_quad<QP_ROT1>(v) : dpp_quad<QP_SWAP2>(v);
  }
}

// sum over the SP lanes of a candidate (bit-identical in all of them)
template <int SP> __device__ __forceinline__ double group_sum(double v) {
  if constexpr (SP == 1) {
    return v;
  } else if constexpr (SP == 2) {
    return v + dpp_quad<QP_SWAP1>(v);
  } else {
    v = v + dpp_quad<QP_SWAP1>(v);
    return v + dpp_quad<QP_SWAP2>(v);
  }
}

// sum over the SF frequency lanes of a candidate (xor butterfly)
__device__ __forceinline__ double freq_sum(double v, int sp, int s_lanes) {
  for (int m = sp; m < s_lanes; m <<= 1) v += __shfl_xor(v, m, WAVE);
  return v;
}

// freq_sum of K values at once.  Each step's exchanges go through the LDS
// crossbar; issued eight at a time, they wait for it once per eight values
// instead of once per value (value by value, the additions and so the
// results are those of freq_sum).
template <int K> __device__ __forceinline__ void freq_sum_n(double *v, int sp, int s_lanes) {
  for (int m = sp; m < s_lanes; m <<= 1) {
#pragma unroll
    for (int e0 = 0; e0 < K; e0 += 8) {
      double o[8];
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (e0 + e < K) o[e] = __shfl_xor(v[e0 + e], m, WAVE);
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (e0 + e < K) v[e0 + e] += o[e];
    }
  }
}

// Compensated accumulation sum += a * b (Kahan's summation with the running
// correction c folded into the product by a fused multiply-add): the error of
// a length-F sum stays at a few units of roundoff of the terms' magnitude
// instead of growing with F.  The true sum is sum - c.
__device__ __forceinline__ void kahan_fma_acc(double &sum, double &c, double a, double b) {
  const double y = __builtin_fma(a, b, -c);
  const double t = sum + y;
  c = (t - sum) - y;
  sum = t;
}

// xor-butterfly of K double-doubles (hi[e] + lo_in[e]) over the SF frequency
// lanes, the exchanges issued together as in freq_sum_n; hi[e] receives the
// sum rounded to a double.  TwoSum's error term does not depend on the
// operand order, so all lanes end with the same bits.
template <int K> __device__ __forceinline__ void freq_sum_dd_n(double *hi, const double *lo_in, int sp, int s_lanes) {
  double lo[K];
#pragma unroll
  for (int e = 0; e < K; ++e) lo[e] = lo_in[e];
  for (int m = sp; m < s_lanes; m <<= 1) {
    double oh[K], ol[K];
#pragma unroll
    for (int e = 0; e < K; ++e) {
      oh[e] = __shfl_xor(hi[e], m, WAVE);
      ol[e] = __shfl_xor(lo[e], m, WAVE);
    }
#pragma unroll
    for (int e = 0; e < K; ++e) {
      const double s = hi[e] + oh[e];
      const double bv = s - hi[e];
      const double se = (hi[e] - (s - bv)) + (oh[e] - bv);
      hi[e] = s;
      lo[e] = (lo[e] + ol[e]) + se;
    }
  }
#pragma unroll
  for (int e = 0; e < K; ++e) hi[e] = hi[e] + lo[e];
}

// --------------------------------------------------------------------------
// Double-double arithmetic for the extended-precision refinement
// (FLAG_DD_REFINE).  A value is an unevaluated sum h + l.  TwoSum (Knuth)
// gives the rounding error of a sum and the fused multiply-add that of a
// product exactly, so sums and products of such pairs keep about 104 bits.
// Contraction is switched off in these routines: a product that the compiler
// fused into a later sum would no longer be the rounded product whose error
// the next operation recovers.
// --------------------------------------------------------------------------
struct ddv {
  double h, l;
};
__device__ __forceinline__ ddv two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b, bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
// valid when |a| >= |b| (or a == 0)
__device__ __forceinline__ ddv quick_two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ ddv dd_mul(ddv a, ddv b) {
#pragma clang fp contract(off)
  const double p = a.h * b.h;
  const double e = __builtin_fma(a.h, b.l, __builtin_fma(a.l, b.h, __builtin_fma(a.h, b.h, -p)));
  return quick_two_sum(p, e);
}
// sum of two pairs whose high parts do not cancel
__device__ __forceinline__ ddv dd_add(ddv a, ddv b) {
#pragma clang fp contract(off)
  const ddv s = two_sum(a.h, b.h);
  return quick_two_sum(s.h, s.l + (a.l + b.l));
}

// 10^t as a double-double, for |t| <= 30 (relative error near 2^-95).  The
// double nearest 10^t is off by up to half an ulp, which moves the weights
// of an ill-conditioned fit, and with them its cost, by more than the cost's
// tolerance; the extended-precision refinement needs the relaxation times
// to its own precision.  Steps: y = t ln 10 in double-double; y = n ln 2 + r
// with n = rint(y / ln 2), |r| <= ln 2 / 2; e^r = (e^(r/256))^256, the inner
// factor from its Taylor series to degree 9 (the first omitted term is below
// 2^-117), the power by eight squarings; then the scale 2^n.
__device__ __noinline__ ddv exp10_dd(double t) {
#pragma clang fp contract(off)
  constexpr double LN10_H = 0x1.26bb1bbb55516p+1, LN10_L = -0x1.f48ad494ea3e9p-53;
  constexpr double LN2_H = 0x1.62e42fefa39efp-1, LN2_L = 0x1.abc9e3b39803fp-56;
  const double yh = t * LN10_H;
  const double yl = __builtin_fma(t, LN10_L, __builtin_fma(t, LN10_H, -yh));
  const double n = rint(yh / LN2_H);
  // r = y - n ln 2: n * LN2_H and its rounding error exactly, then the rest
  const double ph = n * LN2_H;
  const double pe = __builtin_fma(n, LN2_H, -ph);
  ddv r = two_sum(yh, -ph);
  r = quick_two_sum(r.h, r.l + ((yl - pe) - n * LN2_L));
  r.h = ldexp(r.h, -8);
  r.l = ldexp(r.l, -8);
  // 1 + r (1 + r/2 (1 + r/3 ( ... (1 + r/9))))
  ddv p = {1.0, 0.0};
  for (int j = 9; j >= 1; --j) {
    const double dj = (double)j;
    const double qh = r.h / dj;
    const double ql = (__builtin_fma(-qh, dj, r.h) + r.l) / dj;   // the remainder r.h - qh j is exact
    p = dd_add({1.0, 0.0}, dd_mul({qh, ql}, p));
  }
  for (int s = 0; s < 8; ++s) p = dd_mul(p, p);
  const int e = (int)n;
  return {ldexp(p.h, e), ldexp(p.l, e)};
}

// The Debye basis term I = x / (1 + x^2), x = w tau, as a double-double from
// tau = th + tl: x by TwoProduct, x^2 likewise (its cross term 2 xh xl added
// to the error), 1 + x^2 by TwoSum, R = 1 / (1 + x^2) from a reciprocal of
// the high part within half an ulp and one correction r (1 + e), e = 1 - d r
// formed with fused operations, then I = x R.
__device__ __forceinline__ ddv dd_debye_I(double w, double th, double tl) {
#pragma clang fp contract(off)
  const double xh = w * th;
  const double xl = __builtin_fma(w, tl, __builtin_fma(w, th, -xh));
  const double qh = xh * xh;
  const double ql = __builtin_fma(xh + xh, xl, __builtin_fma(xh, xh, -qh));
  const ddv d = two_sum(1.0, qh);
  const double dl = d.l + ql;
  const double r = rcp_nr(d.h);
  const double rl = r * __builtin_fma(-dl, r, __builtin_fma(-d.h, r, 1.0));
  const double ih = xh * r;
  return {ih, __builtin_fma(xh, rl, __builtin_fma(xl, r, __builtin_fma(xh, r, -ih)))};
}

// --------------------------------------------------------------------------
// Debye basis of the owned poles at one frequency: R = 1/(1+x^2), I = x R.
// Every pass needs only R: with I = w tau R, the factor tau moves out of
// every frequency sum (applied once per candidate) and w out of every pole
// sum (applied once per point), and 1 + x^2 is 1 + w^2 tau^2 with w^2 shared
// by the poles and tau^2 by the points (the rounding of d is the same as
// through x = w tau: one product rounded, then a fused add).  Padded poles
// have tau = 0: R = 1, and their I columns vanish through tau.
//
// Paired form (basis_R): two poles share one reciprocal, r = 1/(d0 d1),
// R0 = d1 r, R1 = d0 r (within a few ulp).  With |log10 tau| <= 30 (larger
// values are rejected as bad input) and w < 1e45 rad/s, x < 1e75 and the
// product d0 d1 < 1e301 cannot overflow.
// --------------------------------------------------------------------------
template <int NB>
__device__ __forceinline__ void basis_R(double w2, const double *tau2, double *R) {
#pragma unroll
  for (int c = 0; c + 1 < NB; c += 2) {
    const double d0 = __builtin_fma(w2, tau2[c], 1.0), d1 = __builtin_fma(w2, tau2[c + 1], 1.0);
    const double r = rcp_nr(d0 * d1);
    R[c] = d1 * r;
    R[c + 1] = d0 * r;
  }
  if constexpr (NB & 1) R[NB - 1] = rcp_nr(__builtin_fma(w2, tau2[NB - 1], 1.0));
}

// Grouped form (the frequency passes of the cost): four poles share one
// reciprocal, r = 1/(p01 p23) with p01 = d0 d1, p23 = d2 d3, and
// 1/d0 = d1 (r p23), 1/d1 = d0 (r p23), 1/d2 = d3 (r p01), 1/d3 = d2 (r p01):
// three products and one reciprocal per four poles in place of two
// reciprocals (a reciprocal occupies the FP64 pipe for four issue cycles and
// its Newton step for three more).  Poles beyond the last full group of four
// are paired as above.
//
// The product of four d can leave the double range (each d < 1e150), so a
// group works on d scaled by a power of two s, fixed from the bound
// w < 1e45: s^4 prod d(1e45) <= 2^990 and s >= 2^-253, so every intermediate
// product lies in [2^-1012, 2^990] at every admissible frequency and every
// reciprocal is a normal number.  With tau^2 s in place of tau^2 and s in
// place of 1, every intermediate is the unscaled value times an exact power
// of two (the same roundings, barring underflow of tiny products, which the
// scaled form suffers less); the group's basis values come out divided by
// s, and s is applied with tau after the frequency sums.  Any smaller s of
// the same form down to 2^-253 keeps these bounds, so a wave takes, per
// group index, the smallest s of its lanes: s is then wave-uniform and the
// fused add reads it from a scalar register (a third vector operand of a
// 64-bit FMA costs issue bandwidth), and each lane's results do not depend
// on the other lanes of its wave.
// --------------------------------------------------------------------------
constexpr double OMEGA_BOUND = 1e45;   // admissible angular frequencies: 0 < w < OMEGA_BOUND

template <int NB> struct Groups {
  static constexpr int NQ = NB / 4;              // groups of four owned poles
  static constexpr int NS = NQ > 0 ? NQ : 1;     // (array size)
};

// scale s = 2^-k of each group (from tau^2 of its poles), the same in every
// lane of the wave (all lanes call this together)
template <int NB>
__device__ __forceinline__ void group_scales(const double *tau2, int *kq, double *sq) {
  kq[0] = 0;
  sq[0] = 1.0;
#pragma unroll
  for (int g = 0; g < Groups<NB>::NQ; ++g) {
    int e = 0;   // sum of the binary exponents: prod d(1e45) < 2^e
#pragma unroll
    for (int t = 0; t < 4; ++t)
      e += __builtin_amdgcn_frexp_exp(__builtin_fma(OMEGA_BOUND * OMEGA_BOUND, tau2[4 * g + t], 1.0));
    int k = e > 990 ? (e - 990 + 3) >> 2 : 0;
    // |log10 tau| <= 30 gives e <= 1996, k <= 252; the cap keeps a lane with
    // rejected input (its results are discarded) from scaling its wave's
    // valid lanes out of range
    k = k < 253 ? k : 253;
#pragma unroll
    for (int m = 1; m < WAVE; m <<= 1) {
      const int o = __shfl_xor(k, m, WAVE);
      k = o > k ? o : k;
    }
    k = __builtin_amdgcn_readfirstlane(k);
    kq[g] = k;
    sq[g] = __hiloint2double((1023 - k) << 20, 0);   // 2^-k
  }
}

// scale of owned pole i (1 outside the groups)
template <int NB> __device__ __forceinline__ double pole_scale(const double *sq, int i) {
  return i < 4 * Groups<NB>::NQ ? sq[i / 4] : 1.0;
}

// x * 2^(+-k) of owned pole i's group (exact)
template <int NB> __device__ __forceinline__ double group_unscale(const int *kq, int i, double x) {
  return i < 4 * Groups<NB>::NQ ? __builtin_amdgcn_ldexp(x, kq[i / 4]) : x;
}
template <int NB> __device__ __forceinline__ double group_scale(const int *kq, int i, double x) {
  return i < 4 * Groups<NB>::NQ ? __builtin_amdgcn_ldexp(x, -kq[i / 4]) : x;
}

// R / s of the owned poles (tau2s = tau^2 s)
template <int NB>
__device__ __forceinline__ void basis_Rs(double w2, const double *tau2s, const double *sq, double *R) {
#pragma unroll
  for (int g = 0; g < Groups<NB>::NQ; ++g) {
    const int c = 4 * g;
    const double d0 = __builtin_fma(w2, tau2s[c], sq[g]), d1 = __builtin_fma(w2, tau2s[c + 1], sq[g]);
    const double d2 = __builtin_fma(w2, tau2s[c + 2], sq[g]), d3 = __builtin_fma(w2, tau2s[c + 3], sq[g]);
    const double p01 = d0 * d1, p23 = d2 * d3;
    const double r = rcp_nr(p01 * p23);
    const double r01 = r * p23, r23 = r * p01;
    R[c] = d1 * r01;
    R[c + 1] = d0 * r01;
    R[c + 2] = d3 * r23;
    R[c + 3] = d2 * r23;
  }
  basis_R<NB - 4 * Groups<NB>::NQ>(w2, tau2s + 4 * Groups<NB>::NQ, R + 4 * Groups<NB>::NQ);
}

// U / s with U = w R directly (the Gram pass needs no R): the factor w enters
// after the group's reciprocal is split, U0 = d1 (w (r p23)), ... (r p23 =
// 1/p01 <= 2^506, so no intermediate overflows even where the wave's scale is
// far below the lane's own and r is near 2^1012), and once per pair for the
// paired poles (U0 = d1 (w r)).
template <int NB>
__device__ __forceinline__ void basis_Us(double w, double w2, const double *tau2s, const double *sq, double *U) {
#pragma unroll
  for (int g = 0; g < Groups<NB>::NQ; ++g) {
    const int c = 4 * g;
    const double d0 = __builtin_fma(w2, tau2s[c], sq[g]), d1 = __builtin_fma(w2, tau2s[c + 1], sq[g]);
    const double d2 = __builtin_fma(w2, tau2s[c + 2], sq[g]), d3 = __builtin_fma(w2, tau2s[c + 3], sq[g]);
    const double p01 = d0 * d1, p23 = d2 * d3;
    const double r = rcp_nr(p01 * p23);
    const double r01 = w * (r * p23), r23 = w * (r * p01);
    U[c] = d1 * r01;
    U[c + 1] = d0 * r01;
    U[c + 2] = d3 * r23;
    U[c + 3] = d2 * r23;
  }
  constexpr int C = 4 * Groups<NB>::NQ;
#pragma unroll
  for (int c = C; c + 1 < NB; c += 2) {
    const double d0 = __builtin_fma(w2, tau2s[c], 1.0), d1 = __builtin_fma(w2, tau2s[c + 1], 1.0);
    const double rw = w * rcp_nr(d0 * d1);
    U[c] = d1 * rw;
    U[c + 1] = d0 * rw;
  }
  if constexpr ((NB - C) & 1) U[NB - 1] = w * rcp_nr(__builtin_fma(w2, tau2s[NB - 1], 1.0));
}

// Owned poles left over after the groups of four and the pairs: one (the
// last) or none.
template <int NB> constexpr bool odd_pole() { return ((NB - 4 * Groups<NB>::NQ) & 1) != 0; }

// The basis at two points a and b (w2 = w^2).  With an odd last pole, that
// pole's two values share one reciprocal, r = 1/(d_a d_b), R_a = d_b r,
// R_b = d_a r, as two poles of one point do (the odd pole lies outside the
// groups, so d <= 1e150 and d_a d_b cannot overflow); the other poles as in
// basis_Rs / basis_Us at each point.
template <int NB>
__device__ __forceinline__ void basis_Rs2(double w2a, double w2b, const double *tau2s, const double *sq, double *Ra,
                                          double *Rb) {
  if constexpr (odd_pole<NB>()) {
    basis_Rs<NB - 1>(w2a, tau2s, sq, Ra);
    basis_Rs<NB - 1>(w2b, tau2s, sq, Rb);
    const double da = __builtin_fma(w2a, tau2s[NB - 1], 1.0), db = __builtin_fma(w2b, tau2s[NB - 1], 1.0);
    const double r = rcp_nr(da * db);
    Ra[NB - 1] = db * r;
    Rb[NB - 1] = da * r;
  } else {
    basis_Rs<NB>(w2a, tau2s, sq, Ra);
    basis_Rs<NB>(w2b, tau2s, sq, Rb);
  }
}
template <int NB>
__device__ __forceinline__ void basis_Us2(double wa, double wb, const double *tau2s, const double *sq, double *Ua,
                                          double *Ub) {
  if constexpr (odd_pole<NB>()) {
    basis_Us<NB - 1>(wa, wa * wa, tau2s, sq, Ua);
    basis_Us<NB - 1>(wb, wb * wb, tau2s, sq, Ub);
    const double da = __builtin_fma(wa * wa, tau2s[NB - 1], 1.0), db = __builtin_fma(wb * wb, tau2s[NB - 1], 1.0);
    const double r = rcp_nr(da * db);
    Ua[NB - 1] = wa * (db * r);
    Ub[NB - 1] = wb * (da * r);
  } else {
    basis_Us<NB>(wa, wa * wa, tau2s, sq, Ua);
    basis_Us<NB>(wb, wb * wb, tau2s, sq, Ub);
  }
}

// R / s of the poles of two owner lanes (a half-candidate of the four-lane
// split, a whole candidate of the two-lane split): each owner's NQ groups of
// four at the wave's group scales (t2[0 .. 8 NQ), owner A's groups then
// owner B's, tau^2 s), then their LO leftover poles each (t2[8 NQ ..), tau^2,
// unscaled, so that d <= 1e150) in pairs sharing a reciprocal.
template <int NQ, int LO>
__device__ __forceinline__ void basis_two_owners(double w2, const double *t2, const double *sq, double *R) {
#pragma unroll
  for (int c = 0; c < 8 * NQ; c += 4) {
    const double s = sq[(c / 4) % NQ];
    const double d0 = __builtin_fma(w2, t2[c], s), d1 = __builtin_fma(w2, t2[c + 1], s);
    const double d2 = __builtin_fma(w2, t2[c + 2], s), d3 = __builtin_fma(w2, t2[c + 3], s);
    const double p01 = d0 * d1, p23 = d2 * d3;
    const double r = rcp_nr(p01 * p23);
    const double r01 = r * p23, r23 = r * p01;
    R[c] = d1 * r01;
    R[c + 1] = d0 * r01;
    R[c + 2] = d3 * r23;
    R[c + 3] = d2 * r23;
  }
#pragma unroll
  for (int c = 8 * NQ; c < 8 * NQ + 2 * LO; c += 2) {
    const double d0 = __builtin_fma(w2, t2[c], 1.0), d1 = __builtin_fma(w2, t2[c + 1], 1.0);
    const double r = rcp_nr(d0 * d1);
    R[c] = d1 * r;
    R[c + 1] = d0 * r;
  }
}

// --------------------------------------------------------------------------
// Dense solve helpers on a packed upper triangle held in registers (SP == 1)
// or in LDS (SP > 1).  A = U^T U, U upper, diagonal stored as reciprocals in uinv.
// --------------------------------------------------------------------------
template <int N, class MAT>
__device__ __forceinline__ bool equilibrate_factor(MAT &A, double *invd, double *uinv, double damping,
                                                   double tol) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double g = A[tri(N, i, i)];
    ok = ok && (g > 0.0) && (g < INFINITY);
    invd[i] = 1.0 / sqrt(g);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = i + 1; j < N; ++j) A[tri(N, i, j)] = A[tri(N, i, j)] * invd[i] * invd[j];
    A[tri(N, i, i)] = 1.0 + damping;
  }
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double s = A[tri(N, j, j)];
#pragma unroll
    for (int l = 0; l < j; ++l) s = __builtin_fma(-A[tri(N, l, j)], A[tri(N, l, j)], s);
    ok = ok && (s > tol);
    double u = sqrt(s);
    double ui = 1.0 / u;
    uinv[j] = ui;
    A[tri(N, j, j)] = u;
#pragma unroll
    for (int k = j + 1; k < N; ++k) {
      double t = A[tri(N, j, k)];
#pragma unroll
      for (int l = 0; l < j; ++l) t = __builtin_fma(-A[tri(N, l, j)], A[tri(N, l, k)], t);
      A[tri(N, j, k)] = t * ui;
    }
  }
  return ok;
}

// x <- A^-1 x with A = U^T U (x overwritten)
template <int N, class MAT, class VEC>
__device__ __forceinline__ void chol_solve(const MAT &A, const double *uinv, VEC &x) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double s = x[i];
#pragma unroll
    for (int l = 0; l < i; ++l) s = __builtin_fma(-A[tri(N, l, i)], x[l], s);
    x[i] = s * uinv[i];
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    double s = x[i];
#pragma unroll
    for (int l = i + 1; l < N; ++l) s = __builtin_fma(-A[tri(N, i, l)], x[l], s);
    x[i] = s * uinv[i];
  }
}

// The same factorisation and solves for a matrix in LDS (SP > 1).  Every
// lane of a candidate runs them on that candidate's region.  The pointers are
// typed as LDS (address space 3): through a generic pointer the calls would
// read with flat loads, whose latency each step of these serial recurrences
// waits for.  The upper triangle is packed by columns (element (i, j), i <= j,
// at j (j + 1) / 2 + i), so that every inner sum of the factorisation and of
// the forward solve reads consecutive elements: one base address and
// immediate offsets, no per-term address arithmetic.  Those sums are unrolled
// by four (their loads issued together, the additions in their order); the
// backward solve is unrolled whole (all its addresses are constants).  The
// operations and their order are those of the register form above.
using lds_ptr = __attribute__((address_space(3))) double *;
using lds_cptr = const __attribute__((address_space(3))) double *;

constexpr __host__ __device__ int tcol(int i, int j) { return j * (j + 1) / 2 + i; }

template <int N>
__device__ __noinline__ bool lds_equilibrate_factor(lds_ptr A, lds_ptr invd, lds_ptr uinv, double damping,
                                                    double tol) {
  bool ok = true;
  double dv[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double g = A[tcol(i, i)];
    ok = ok && (g > 0.0) && (g < INFINITY);
    dv[i] = 1.0 / sqrt(g);
    invd[i] = dv[i];
  }
#pragma unroll
  for (int j = 0; j < N; ++j) {
#pragma unroll
    for (int i = 0; i < j; ++i) A[tcol(i, j)] = A[tcol(i, j)] * dv[i] * dv[j];
    A[tcol(j, j)] = 1.0 + damping;
  }
  for (int j = 0; j < N; ++j) {
    const lds_ptr cj = A + tcol(0, j);
    double s = cj[j];
#pragma unroll 4
    for (int l = 0; l < j; ++l) s = __builtin_fma(-cj[l], cj[l], s);
    ok = ok && (s > tol);
    const double u = sqrt(s);
    const double ui = 1.0 / u;
    uinv[j] = ui;
    cj[j] = u;
    for (int k = j + 1; k < N; ++k) {
      const lds_ptr ck = A + tcol(0, k);
      double t = ck[j];
#pragma unroll 4
      for (int l = 0; l < j; ++l) t = __builtin_fma(-cj[l], ck[l], t);
      ck[j] = t * ui;
    }
  }
  return ok;
}

template <int N> __device__ __noinline__ void lds_chol_solve(lds_cptr A, lds_cptr uinv, lds_ptr x) {
  double xv[N];
  for (int i = 0; i < N; ++i) {
    const lds_cptr ci = A + tcol(0, i);
    double s = x[i];
#pragma unroll 4
    for (int l = 0; l < i; ++l) s = __builtin_fma(-ci[l], x[l], s);
    x[i] = s * uinv[i];
  }
#pragma unroll
  for (int i = 0; i < N; ++i) xv[i] = x[i];
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    double s = xv[i];
#pragma unroll
    for (int l = i + 1; l < N; ++l) s = __builtin_fma(-A[tcol(i, l)], xv[l], s);
    xv[i] = s * uinv[i];
    x[i] = xv[i];
  }
}

// per-candidate LDS region of the SP > 1 path: packed triangle, then five
// vectors of N (scaling, reciprocal pivots, rhs, two work vectors)
template <int N> struct LdsLayout {
  static constexpr int NT = N * (N + 1) / 2;
  static constexpr int DOUBLES = NT + 5 * N;
  double *A, *invd, *uinv, *vb, *vz, *vw;
  __device__ __forceinline__ explicit LdsLayout(double *base)
      : A(base), invd(base + NT), uinv(base + NT + N), vb(base + NT + 2 * N), vz(base + NT + 3 * N),
        vw(base + NT + 4 * N) {}
};

// factor parked by the SP == 1 path: A (off-diagonal) and reciprocal pivots
template <int N>
__device__ __forceinline__ void unpark(const double *park, int cpw, int grp, double *A, double *uinv) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      const double v = park[tri(N, i, j) * cpw + grp];
      if (i == j) uinv[i] = v;
      else A[tri(N, i, j)] = v;
    }
}

// --------------------------------------------------------------------------
// Cost pass in rational form.  With w >= 0 (the sign flip) the model sums
// over a set of NR poles are rational functions of y = w^2 with positive
// coefficients,
//   sum_i w_i R_i = P(y) / Q(y),  sum_i (w_i tau_i) R_i = P'(y) / Q(y),
//   Q(y) = prod_i (1 + y tau_i^2),  P(y) = sum_i w_i prod_{j != i} (1 + y tau_j^2),
// evaluated by Horner's rule with one reciprocal per point (no cancellation:
// every term is positive).  The variable is scaled by the largest tau^2 of
// the set, so every coefficient is at most binomial-sized.  GS lanes, each
// with its own set, add their sums at every point (GS = 1: the set is the
// whole candidate).  The lane takes points k0, k0 + stride, ... and returns
// its partial sums of squared residuals (cost) and of eps' - shift - model
// (sa).  Returns true when the wave must use the basis form instead: a
// lane's smallest coefficient would be subnormal, Q exceeds 1e280 at some
// point, or a cost is not finite (lanes that do not matter are ignored).
// --------------------------------------------------------------------------
template <int NR, int GS, class LOAD, class LOAD_FIRST>
__device__ __forceinline__ bool rational_cost_pass(const double *tau2, const double *w, const double *wt,
                                                   bool matters, int64_t k0, int64_t stride, int64_t F,
                                                   const double *om, const double *epr, const double *epi,
                                                   double shift, LOAD ld, LOAD_FIRST ld_first, double &cost,
                                                   double &sa) {
  double tmax = 0.0;
#pragma unroll
  for (int i = 0; i < NR; ++i) tmax = tau2[i] > tmax ? tau2[i] : tmax;
  const double isc = tmax > 0.0 ? 1.0 / tmax : 1.0;
  // coefficients built one pole at a time, every update a sum of positive
  // terms: with t the pole's scaled tau^2,
  //   P <- P (1 + y t) + w Q,  P' <- P' (1 + y t) + (w tau) Q,  Q <- Q (1 + y t)
  // (O(NR^2) fused multiply-adds; only Q, P, P' stay live)
  double qc[NR + 1], cr[NR], ci[NR];
  double pnz = 1.0;   // product of the nonzero scaled tau^2: the smallest coefficient
  qc[0] = 1.0;
#pragma unroll
  for (int k = 1; k <= NR; ++k) qc[k] = 0.0;
#pragma unroll
  for (int k = 0; k < NR; ++k) cr[k] = ci[k] = 0.0;
#pragma unroll
  for (int m = 0; m < NR; ++m) {
    const double t = tau2[m] * isc, wm = w[m], wtm = wt[m];
    pnz *= t > 0.0 ? t : 1.0;
#pragma unroll
    for (int k = m; k >= 1; --k) {
      cr[k] = __builtin_fma(wm, qc[k], __builtin_fma(t, cr[k - 1], cr[k]));
      ci[k] = __builtin_fma(wtm, qc[k], __builtin_fma(t, ci[k - 1], ci[k]));
    }
    cr[0] = __builtin_fma(wm, qc[0], cr[0]);
    ci[0] = __builtin_fma(wtm, qc[0], ci[0]);
#pragma unroll
    for (int k = m + 1; k >= 1; --k) qc[k] = __builtin_fma(t, qc[k - 1], qc[k]);
  }
  double csum = qc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) csum += cr[k] + ci[k];
  const bool coef_ok = !matters || (pnz >= 1e-280 && fabs(csum) < INFINITY);
  if (__builtin_amdgcn_ballot_w64(!coef_ok) != 0) return true;
  cost = 0.0;
  sa = 0.0;
  double qmax = 0.0;
  int64_t k = k0;
  double w_n = 0, er_n = 0, ei_n = 0;
  if (k < F) {
    w_n = ld_first(om, k);
    er_n = ld_first(epr, k);
    ei_n = ld_first(epi, k);
  }
  // two points per trip: their Horner and reciprocal chains interleave
#pragma unroll 2
  for (; k < F; k += stride) {
    const double om_k = w_n, er = er_n, ei = ei_n;
    const int64_t kn = (k + stride < F) ? k + stride : k;   // in-bounds prefetch, no branch
    w_n = ld(om, kn);
    er_n = ld(epr, kn);
    ei_n = ld(epi, kn);
    const double y = (om_k * om_k) * tmax;
    double hq = qc[NR], hr = cr[NR - 1], hi = ci[NR - 1];
#pragma unroll
    for (int d = NR - 1; d >= 0; --d) hq = __builtin_fma(hq, y, qc[d]);
#pragma unroll
    for (int d = NR - 2; d >= 0; --d) {
      hr = __builtin_fma(hr, y, cr[d]);
      hi = __builtin_fma(hi, y, ci[d]);
    }
    qmax = hq > qmax ? hq : qmax;
    const double r = rcp_nr(hq);
    const double rr = (er - shift) - group_sum<GS>(hr * r);
    const double ri = __builtin_fma(-om_k, group_sum<GS>(hi * r), ei);
    sa += rr;
    cost = __builtin_fma(rr, rr, cost);
    cost = __builtin_fma(ri, ri, cost);
  }
  return __builtin_amdgcn_ballot_w64(matters && (!(qmax <= 1e280) || !(fabs(cost) + fabs(sa) < INFINITY))) != 0;
}

// --------------------------------------------------------------------------
// The kernel.  GRAD adds the adjoint (grad w.r.t. log10 tau, and per-candidate
// records for the target gradient).
// --------------------------------------------------------------------------
// target waves per SIMD: bounds the register budget of each instantiation
// (three for the small one-lane kernels, which fit 168 registers; two
// elsewhere: the N = 12 two-lane kernels fit three waves with one point per
// trip of the Gram pass, but two waves with two points per trip are faster)
template <int N, int SP, bool GRAD, int UNI> constexpr int waves_per_simd() {
  return (SP == 1 && N <= 6) ? 3 : 2;
}

// UNI (uniform tiles; the plan checks that every active lane of every tile
// belongs to one material and that spectra hold fewer than 2^29 points):
//   1: frequency split 1, so every lane of a wave reads the same point and
//      the spectra are read with wave-uniform (scalar) loads;
//   2: frequency split > 1: wave-uniform spectrum base, per-lane 32-bit
//      byte offsets (one offset per point for the three arrays).
// XR: the refinement pass in double-double (FLAG_DD_REFINE; forward only).
// One work tile (one wavefront: the candidates the plan lists for it) of the
// cost kernel for N poles; the kernels below call it for their tiles.
template <int N, int SP, bool GRAD, int UNI, bool XR = false>
__device__ __forceinline__ void fit_tile(const FitArgs &a, const int64_t tile) {
  static_assert(!(XR && GRAD), "the extended-precision refinement is a forward-kernel form");
  using S = Shape<N, SP>;
  constexpr int NB = S::NB, NV = S::NV, NG = S::NG, D = S::D;
  extern __shared__ double lds_all[];

  const int lane = threadIdx.x;
  const int SF = UNI == 1 ? 1 : a.freq_split;
  const int SL = SP * SF;            // lanes per candidate
  const int grp = lane / SL;         // candidate slot in the wave
  const int sub = lane - grp * SL;
  const int q = sub % SP;            // pole block
  const int fl = UNI == 1 ? 0 : sub / SP; // frequency lane
  const int64_t slot = tile * a.cand_per_wave + grp;
  const int32_t cand = a.lane_cand[slot];
  const bool active = cand >= 0;
  const int32_t mat = active ? a.lane_mat[slot] : 0;
  const int64_t c = active ? cand : 0;
  // a wave whose candidates all belong to materials marked done exits
  // before any work (wave-uniform: a block is one wave)
  if (a.skip_mat && __builtin_amdgcn_ballot_w64(active && a.skip_mat[mat] == 0) == 0) return;

  int64_t f0 = 0, F = 0;
  if constexpr (UNI != 0) {
    const int32_t mu = __builtin_amdgcn_readfirstlane(a.lane_mat[tile * a.cand_per_wave]);
    f0 = a.f_off[mu];
    F = a.f_off[mu + 1] - f0;
  } else if (active) {
    f0 = a.f_off[mat];
    F = a.f_off[mat + 1] - f0;
  }
  const double *om = a.omega + f0;
  const double *epr = a.eps_re + f0;
  const double *epi = a.eps_im + f0;
  // point k of a spectrum
  auto ld = [](const double *p, int64_t k) -> double {
    if constexpr (UNI == 2) return *(const double *)((const char *)p + ((uint32_t)k << 3));
    else return p[k];
  };
  // The first point of a pass that prefetches one point ahead, read through
  // the constant address space (the spectra are read-only during a launch).
  // Loads from two address spaces are not merged, so the compiler keeps the
  // loop's loads one point ahead instead of folding them with this one into a
  // single load at the top of every trip (which would expose the load
  // latency at each point).
  auto ld_first = [](const double *p, int64_t k) -> double {
    using cptr = const __attribute__((address_space(4))) double *;
    if constexpr (UNI == 2) return *(cptr)((const char *)p + ((uint32_t)k << 3));
    else return ((cptr)p)[k];
  };

  const double damping = a.damping;
  const bool flip = !(a.flags & FLAG_NO_SIGN_FLIP);

  // ---- relaxation times of the owned poles
  double tau[NB];
  bool bad = false;
#pragma unroll
  for (int cI = 0; cI < NB; ++cI) {
    const int p = q * NB + cI;
    tau[cI] = 0.0;
    if (p < N && active) {
      const double t = a.theta[c * a.ld + p];
      bad = bad || !(fabs(t) <= THETA_LIMIT);
      tau[cI] = exp10(t);
    }
  }
  // Grouped basis of the frequency passes: group scales s = 2^-k, tau^2 s,
  // and tau s (the factor applied after the sums).  Only these are kept;
  // tau and tau^2 are recovered exactly where needed (ldexp by k).
  int kq[Groups<NB>::NS];
  double sq[Groups<NB>::NS], tau2s[NB], ts[NB];
  {
    double tau2[NB];
#pragma unroll
    for (int cI = 0; cI < NB; ++cI) tau2[cI] = tau[cI] * tau[cI];
    group_scales<NB>(tau2, kq, sq);
#pragma unroll
    for (int cI = 0; cI < NB; ++cI) {
      tau2s[cI] = group_scale<NB>(kq, cI, tau2[cI]);
      ts[cI] = group_scale<NB>(kq, cI, tau[cI]);
    }
  }
  auto tau_of = [&](int cI) { return group_unscale<NB>(kq, cI, ts[cI]); };
  auto tau2_of = [&](int cI) { return group_unscale<NB>(kq, cI, tau2s[cI]); };

  // ---- pass 1: Gram, right-hand side, sum of eps'.  Accumulated with
  // U / s = w R / s in place of I = tau U; the factors tau s are applied
  // after the frequency sums.  (The adjoint's column sums of R, which it needs
  // for eps_inf before its pass 3, are taken in pass 2, which forms every R
  // anyway; the forward kernels take eps_inf from the cost pass.)
  double G[NG], bv[NB], Sv[NB];
#pragma unroll
  for (int e = 0; e < NG; ++e) G[e] = 0.0;
#pragma unroll
  for (int cI = 0; cI < NB; ++cI) {
    bv[cI] = 0.0;
    Sv[cI] = 0.0;
  }
  double sum_er = 0.0;
  // one point of the Gram pass
  // one point of the Gram pass, from its basis values Iv[0 .. NB-1]
  auto gram_acc = [&](double *Iv, double er, double ei) {
#pragma unroll
    for (int cI = 0; cI < NB; ++cI) bv[cI] = __builtin_fma(Iv[cI], ei, bv[cI]);
    if constexpr (SP > 1) {
#pragma unroll
      for (int v = NB; v < NV; ++v) Iv[v] = ring_fetch<SP>(Iv[v % NB], v / NB);
#pragma unroll
      for (int cI = 0; cI < NB; ++cI)
#pragma unroll
        for (int d = 0; d <= D; ++d) G[cI * (D + 1) + d] = __builtin_fma(Iv[cI], Iv[cI + d], G[cI * (D + 1) + d]);
    } else {
#pragma unroll
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = i; j < N; ++j) G[tri(N, i, j)] = __builtin_fma(Iv[i], Iv[j], G[tri(N, i, j)]);
    }
    sum_er += er;
  };
  auto gram_point = [&](double w, double er, double ei) {
    double Iv[NV];
    basis_Us<NB>(w, w * w, tau2s, sq, Iv);
    gram_acc(Iv, er, ei);
  };
  // Two points per trip let the reciprocal chains of their bases interleave.
  // With no DPP in the body (SP == 1) the compiler pairs the points itself.
  // The ring's DPP moves are convergent operations, which the compiler does
  // not unroll into a loop with a remainder, so on the pole-split path the
  // pair is written out where it fits the register budget at two waves per
  // SIMD: four pole lanes up to N = 20 (228 VGPRs at N = 20), two up to
  // N = 14 (the general-tile form from N = 13 on, N = 15, 16 and N > 20
  // spill with it).
  constexpr bool PAIR_RING = (SP == 4 && N <= 20) || (SP == 2 && (N == 12 || (N <= 14 && UNI != 0)));
  if constexpr (!PAIR_RING) {
    int64_t k = fl;
    double w_n = 0, er_n = 0, ei_n = 0;
    if (k < F) {
      w_n = ld_first(om, k);
      er_n = ld_first(epr, k);
      ei_n = ld_first(epi, k);
    }
#pragma unroll SP == 1 ? 2 : 1
    for (; k < F; k += SF) {
      const double w = w_n, er = er_n, ei = ei_n;
      const int64_t kn = (k + SF < F) ? k + SF : k;   // in-bounds prefetch, no branch
      w_n = ld(om, kn);
      er_n = ld(epr, kn);
      ei_n = ld(epi, kn);
      double Iv[NV];
      basis_Us<NB>(w, w * w, tau2s, sq, Iv);
#pragma unroll
      for (int cI = 0; cI < NB; ++cI) bv[cI] = __builtin_fma(Iv[cI], ei, bv[cI]);
      if constexpr (SP > 1) {
#pragma unroll
        for (int v = NB; v < NV; ++v) Iv[v] = ring_fetch<SP>(Iv[v % NB], v / NB);
#pragma unroll
        for (int cI = 0; cI < NB; ++cI)
#pragma unroll
          for (int d = 0; d <= D; ++d) G[cI * (D + 1) + d] = __builtin_fma(Iv[cI], Iv[cI + d], G[cI * (D + 1) + d]);
      } else {
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
          for (int j = i; j < N; ++j) G[tri(N, i, j)] = __builtin_fma(Iv[i], Iv[j], G[tri(N, i, j)]);
      }
      sum_er += er;
    }
  } else {
    // the odd point last; the pole lanes of a candidate share their
    // frequency lane, hence their trip counts
    int64_t k = fl;
    double wa_n = 0, era_n = 0, eia_n = 0, wb_n = 0, erb_n = 0, eib_n = 0;
    if (k < F) {
      wa_n = ld_first(om, k);
      era_n = ld_first(epr, k);
      eia_n = ld_first(epi, k);
    }
    if (k + SF < F) {
      wb_n = ld_first(om, k + SF);
      erb_n = ld_first(epr, k + SF);
      eib_n = ld_first(epi, k + SF);
    }
    for (; k + SF < F; k += 2 * SF) {
      const double wa = wa_n, era = era_n, eia = eia_n, wb = wb_n, erb = erb_n, eib = eib_n;
      // in-bounds prefetch of the next two points, no branch
      const int64_t ka = (k + 2 * SF < F) ? k + 2 * SF : k, kb = (k + 3 * SF < F) ? k + 3 * SF : k;
      wa_n = ld(om, ka);
      era_n = ld(epr, ka);
      eia_n = ld(epi, ka);
      wb_n = ld(om, kb);
      erb_n = ld(epr, kb);
      eib_n = ld(epi, kb);
      double Ia[NV], Ib[NV];
      basis_Us2<NB>(wa, wb, tau2s, sq, Ia, Ib);
      gram_acc(Ia, era, eia);
      gram_acc(Ib, erb, eib);
    }
    if (k < F) gram_point(wa_n, era_n, eia_n);
  }
  freq_sum_n<NG>(G, SP, SL);
  if constexpr (SP > 1) {
    double tv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) tv[v] = v < NB ? ts[v] : ring_fetch<SP>(ts[v % NB], v / NB);
#pragma unroll
    for (int cI = 0; cI < NB; ++cI)
#pragma unroll
      for (int d = 0; d <= D; ++d) G[cI * (D + 1) + d] *= ts[cI] * tv[cI + d];
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = i; j < N; ++j) G[tri(N, i, j)] *= ts[i] * ts[j];
  }
  freq_sum_n<NB>(bv, SP, SL);
#pragma unroll
  for (int cI = 0; cI < NB; ++cI) {
    bv[cI] = bv[cI] * ts[cI];
    bad = bad || !(fabs(bv[cI]) < INFINITY);
  }
  sum_er = freq_sum(sum_er, SP, SL);
  bad = bad || !(fabs(sum_er) < INFINITY);
  bad = group_sum<SP>(bad ? 1.0 : 0.0) != 0.0;

  // ---- DLS solve (equilibrated, damped Cholesky)
  const double tol = 8.0 * (double)(F > N ? F : N) * 0x1.0p-53;
  double zt[NB], zc[NB], invd_own[NB];
  bool ok;
  double *L = nullptr;
  double uinv_r[SP == 1 ? N : 1], invd_r[SP == 1 ? N : 1];
  if constexpr (SP == 1) {
    ok = equilibrate_factor<N>(G, invd_r, uinv_r, damping, tol);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      zt[i] = bv[i] * invd_r[i];
      invd_own[i] = invd_r[i];
    }
    chol_solve<N>(G, uinv_r, zt);
    // Park the factor in LDS (reciprocal pivots in place of its diagonal,
    // which the solves never read), element-major so that a wave's lanes touch
    // consecutive addresses.  The later solves read it back; meanwhile its
    // registers serve the frequency passes.
    {
      double *park = lds_all;
      const int cpw = WAVE / SL;
      if (fl == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
          for (int j = i; j < N; ++j) park[tri(N, i, j) * cpw + grp] = (i == j) ? uinv_r[i] : G[tri(N, i, j)];
      }
      __syncthreads();
    }
  } else {
    // assemble the packed triangle in LDS (all lanes of a candidate write the same values)
    L = lds_all + (int64_t)grp * S::LDS_DOUBLES;
    const LdsLayout<N> lay(L);
    double *A = lay.A, *invd = lay.invd, *uinv = lay.uinv, *vb = lay.vb, *vz = lay.vz;
#pragma unroll
    for (int cI = 0; cI < NB; ++cI) {
      const int p1 = q * NB + cI;
#pragma unroll
      for (int d = 0; d <= D; ++d) {
        int p2 = p1 + d;
        if (p2 >= S::NP) p2 -= S::NP;
        if (p1 < N && p2 < N) {
          const int i = p1 < p2 ? p1 : p2, j = p1 < p2 ? p2 : p1;
          A[tcol(i, j)] = G[cI * (D + 1) + d];
        }
      }
      if (p1 < N) vb[p1] = bv[cI];
    }
    __syncthreads();
    ok = lds_equilibrate_factor<N>((lds_ptr)A, (lds_ptr)invd, (lds_ptr)uinv, damping, tol);
    for (int i = 0; i < N; ++i) vz[i] = vb[i] * invd[i];
    lds_chol_solve<N>((lds_cptr)A, (lds_cptr)uinv, (lds_ptr)vz);
    __syncthreads();
#pragma unroll
    for (int cI = 0; cI < NB; ++cI) {
      const int p = q * NB + cI;
      zt[cI] = p < N ? vz[p] : 0.0;
      invd_own[cI] = p < N ? invd[p] : 0.0;
    }
  }
#pragma unroll
  for (int cI = 0; cI < NB; ++cI) zc[cI] = zt[cI] * invd_own[cI];

  // ---- pass 2: corrected semi-normal equations, g = I^T (eps'' - I z).
  // The residual is nearly orthogonal to the columns of I, so g is a sum with
  // heavy cancellation; it is accumulated with compensation (residual
  // refinement with the residual products summed in extra precision).
  // FLAG_NO_REFINE skips it (the forward kernels skip the whole pass; the
  // adjoint still runs it for the column sums of R that its eps_inf needs).
  const bool refine = XR || !(a.flags & FLAG_NO_REFINE);
  double gv[NB], gl[NB];
#pragma unroll
  for (int cI = 0; cI < NB; ++cI) {
    gv[cI] = 0.0;
    gl[cI] = 0.0;
  }
  if constexpr (XR) {
    // The same g = I^T (eps'' - I z) with every quantity that the rounding
    // of the FP64 pass disturbs carried in double-double: the relaxation
    // times, x = w tau, 1 + x^2, R = 1/(1 + x^2) and I = x R, the residual
    // (its pole sum by TwoSum, the low parts added plainly) and the sums of
    // I r (likewise).  Written with contraction off: every product whose
    // rounding error is recovered must stay a separate rounded product.
#pragma clang fp contract(off)
    double th[NB], tl[NB];
#pragma unroll
    for (int cI = 0; cI < NB; ++cI) {
      const int p = q * NB + cI;
      th[cI] = 0.0;   // padded poles: x = 0, so I = 0
      tl[cI] = 0.0;
      if (p < N && active) {
        const double t = a.theta[c * a.ld + p];
        const ddv v = exp10_dd(fabs(t) <= THETA_LIMIT ? t : 0.0);   // rejected candidates: any finite value
        th[cI] = v.h;
        tl[cI] = v.l;
      }
    }
    if (fl < F) {
      double wn = ld(om, fl), en = ld(epi, fl);
      for (int64_t k = fl; k < F; k += SF) {
        const double w = wn, ei = en;
        const int64_t kn = k + SF < F ? k + SF : k;   // the next point, loaded one trip ahead
        wn = ld(om, kn);
        en = ld(epi, kn);
        double Ih[NB], Il[NB];
        double sh = 0.0, sl = 0.0;   // sum over the owned poles of z_i I_i
#pragma unroll
        for (int cI = 0; cI < NB; ++cI) {
          const ddv I = dd_debye_I(w, th[cI], tl[cI]);
          Ih[cI] = I.h;
          Il[cI] = I.l;
          const double ih = I.h;
          const double ph = zc[cI] * ih;
          const double pl = __builtin_fma(zc[cI], Il[cI], __builtin_fma(zc[cI], ih, -ph));
          const ddv s2 = two_sum(sh, ph);
          sh = s2.h;
          sl = sl + (s2.l + pl);
        }
        if constexpr (SP > 1) {
          // over the candidate's pole lanes (TwoSum's error does not depend
          // on the operand order: every lane ends with the same pair)
          ddv s2 = two_sum(sh, dpp_quad<QP_SWAP1>(sh));
          sl = (sl + dpp_quad<QP_SWAP1>(sl)) + s2.l;
          sh = s2.h;
          if constexpr (SP == 4) {
            s2 = two_sum(sh, dpp_quad<QP_SWAP2>(sh));
            sl = (sl + dpp_quad<QP_SWAP2>(sl)) + s2.l;
            sh = s2.h;
          }
        }
        ddv rr = two_sum(ei, -sh);
        rr = two_sum(rr.h, rr.l - sl);
#pragma unroll
        for (int cI = 0; cI < NB; ++cI) {
          const double gh = Ih[cI] * rr.h;
          const double ge = __builtin_fma(Ih[cI], rr.l, __builtin_fma(Il[cI], rr.h, __builtin_fma(Ih[cI], rr.h, -gh)));
          const ddv s2 = two_sum(gv[cI], gh);
          gv[cI] = s2.h;
          gl[cI] = gl[cI] + (s2.l + ge);
        }
      }
    }
    freq_sum_dd_n<NB>(gv, gl, SP, SL);
  } else if constexpr (!GRAD && (SP == 4 || (SP == 2 && NB <= 6))) {
    if (refine) {
      // The pole splits run this pass over pairs of owner lanes: lane q takes
      // the poles of owner lanes 2h and 2h + 1 (their groups of four, then
      // their leftover poles) on every other point of its frequency lane's
      // points.  On the four-lane split h = q & 1 and the point subset is
      // q >> 1, so a point's model sum needs one exchange (between the two
      // halves) instead of two; on the two-lane split h = 0, the subset is q,
      // and a lane holds the whole candidate: no exchange.  Each point's
      // basis is formed by half the lanes.  The owners' tau^2 s and tau s z
      // reach the lanes through the candidate's LDS region (its
      // right-hand-side and correction vectors are free during this pass),
      // and the sums of (R / s)(w r), added over the point subsets and
      // frequency lanes, return to the owners the same way.  (On the
      // two-lane split only up to N = 12: beyond, its 2 NB poles per lane
      // spill registers.)
      constexpr int NQ = Groups<NB>::NQ;   // groups of four per owner
      constexpr int LO = NB - 4 * NQ;      // leftover poles per owner
      constexpr int H = 2 * NB;            // poles per lane
      constexpr int HP = SP / 2;           // owner pairs per candidate
      const int h = q % HP;
      // the pole of element e: owner 2h's groups, owner 2h + 1's, then owner
      // 2h's leftovers, owner 2h + 1's
      auto pole = [&](int e) -> int {
        const int own = 2 * h + (e < 8 * NQ ? e / (4 * NQ) : (e - 8 * NQ) / (LO > 0 ? LO : 1));
        const int cI = e < 8 * NQ ? e % (4 * NQ) : 4 * NQ + (e - 8 * NQ) % (LO > 0 ? LO : 1);
        return own * NB + cI;
      };
      const LdsLayout<N> lay(L);
      double *st2 = lay.vb, *stz = lay.vw;
#pragma unroll
      for (int cI = 0; cI < NB; ++cI) {
        const int p = q * NB + cI;
        if (p < N) {   // (every frequency lane of the owner writes the same values)
          st2[p] = tau2s[cI];
          stz[p] = zc[cI] * ts[cI];
        }
      }
      __syncthreads();
      double t2h[H], zh[H];
#pragma unroll
      for (int e = 0; e < H; ++e) {
        const int p = pole(e);
        t2h[e] = p < N ? st2[p] : 0.0;   // padded poles: no weight
        zh[e] = p < N ? stz[p] : 0.0;
      }
      double gh[H], gc[H];
#pragma unroll
      for (int e = 0; e < H; ++e) gh[e] = gc[e] = 0.0;
      // four points of the lane at a time (on the four-lane split the two
      // halves of a point subset take the same points, so their exchanges
      // pair up), compensated as below
      const int64_t s2 = 2 * (int64_t)SF;
      // w r at point kk, with the point's R / s in R
      auto pair_resid = [&](int64_t kk, double *R) {
        const double w = ld(om, kk);
        basis_two_owners<NQ, LO>(w * w, t2h, sq, R);
        double part = 0.0;
#pragma unroll
        for (int e = 0; e < H; ++e) part = __builtin_fma(R[e], zh[e], part);
        if constexpr (HP == 2) part = part + dpp_quad<QP_SWAP1>(part);
        return w * __builtin_fma(-w, part, ld(epi, kk));
      };
      auto blk = [&](int64_t k0, int np) {   // np >= 1 points
        double pb[H], R[H];
        {
          const double wr = pair_resid(k0, R);
#pragma unroll
          for (int e = 0; e < H; ++e) pb[e] = R[e] * wr;
        }
        for (int t = 1; t < np; ++t) {
          const double wr = pair_resid(k0 + t * s2, R);
#pragma unroll
          for (int e = 0; e < H; ++e) pb[e] = __builtin_fma(R[e], wr, pb[e]);
        }
#pragma unroll
        for (int e = 0; e < H; ++e) kahan_fma_acc(gh[e], gc[e], 1.0, pb[e]);
      };
      // (two blocks per trip, so that the compensated sums alternate between
      // two registers instead of being copied back every update)
      int64_t k = (q / HP) * SF + fl;
      for (; k + 7 * s2 < F; k += 8 * s2) {
        blk(k, 4);
        blk(k + 4 * s2, 4);
      }
      if (k + 3 * s2 < F) {
        blk(k, 4);
        k += 4 * s2;
      }
      if (k < F) blk(k, (int)((F - 1 - k) / s2) + 1);
      {
        double ngc[H];
#pragma unroll
        for (int e = 0; e < H; ++e) ngc[e] = -gc[e];
        freq_sum_dd_n<H>(gh, ngc, HP, SL);   // the point subsets and the frequency lanes
      }
      __syncthreads();
#pragma unroll
      for (int e = 0; e < H; ++e) {
        const int p = pole(e);
        if (p < N) st2[p] = gh[e];   // (both point subsets hold the same sums)
      }
      __syncthreads();
#pragma unroll
      for (int cI = 0; cI < NB; ++cI) {
        const int p = q * NB + cI;
        gv[cI] = (p < N ? st2[p] : 0.0) * ts[cI];
      }
    }
  } else if (GRAD || refine) {
    // I z = w sum_i (tau_i s_i z_i) (R_i / s_i), and I^T r = tau s ((R / s)^T (w r))
    double zs[NB];
#pragma unroll
    for (int cI = 0; cI < NB; ++cI) zs[cI] = zc[cI] * ts[cI];
    // R / s at point k (for the adjoint its column sums taken on the way) and w_k r_k
    // w_k r_k from the basis values Rv at point k (for the adjoint the column
    // sums of R taken on the way)
    auto resid_R = [&](double w, double ei, const double *Rv) {
      double part = 0.0;
#pragma unroll
      for (int cI = 0; cI < NB; ++cI) {
        if constexpr (GRAD) Sv[cI] += Rv[cI];
        part = __builtin_fma(Rv[cI], zs[cI], part);
      }
      return w * __builtin_fma(-w, group_sum<SP>(part), ei);
    };
    auto resid = [&](double w, double ei, double *Rv) {
      basis_Rs<NB>(w * w, tau2s, sq, Rv);
      return resid_R(w, ei, Rv);
    };
    // The compensated sum takes the terms of four points at a time, summed
    // plainly (at most four roundings of terms of the same four points, so
    // the error bound stays a small multiple of the roundoff of the terms'
    // magnitudes; a CPU emulation of the whole solve put the cost error
    // against the 80-bit oracle at the level of single-term compensation).
    auto block4 = [&](int64_t k0) {
      double pb[NB];
      if constexpr (odd_pole<NB>() && SP == 4) {
        // the points in pairs: the odd pole's values of two points share a
        // reciprocal (the terms and their order as below; on the four-lane
        // split only, where the extra registers are free: with one lane per
        // candidate they spill)
#pragma unroll
        for (int t = 0; t < 4; t += 2) {
          const int64_t ka = k0 + t * SF, kb = ka + SF;
          const double wa = ld(om, ka), wb = ld(om, kb);
          double Ra[NB], Rb[NB];
          basis_Rs2<NB>(wa * wa, wb * wb, tau2s, sq, Ra, Rb);
          const double wra = resid_R(wa, ld(epi, ka), Ra);
#pragma unroll
          for (int cI = 0; cI < NB; ++cI) pb[cI] = t == 0 ? Ra[cI] * wra : __builtin_fma(Ra[cI], wra, pb[cI]);
          const double wrb = resid_R(wb, ld(epi, kb), Rb);
#pragma unroll
          for (int cI = 0; cI < NB; ++cI) pb[cI] = __builtin_fma(Rb[cI], wrb, pb[cI]);
        }
      } else {
        double R[NB];
        {
          const double wr = resid(ld(om, k0), ld(epi, k0), R);
#pragma unroll
          for (int cI = 0; cI < NB; ++cI) pb[cI] = R[cI] * wr;
        }
#pragma unroll
        for (int t = 1; t < 4; ++t) {
          const int64_t kk = k0 + t * SF;
          const double wr = resid(ld(om, kk), ld(epi, kk), R);
#pragma unroll
          for (int cI = 0; cI < NB; ++cI) pb[cI] = __builtin_fma(R[cI], wr, pb[cI]);
        }
      }
#pragma unroll
      for (int cI = 0; cI < NB; ++cI) kahan_fma_acc(gv[cI], gl[cI], 1.0, pb[cI]);
    };
    // two blocks per trip: the compensated sums then alternate between two
    // registers instead of being copied back every update
    int64_t k = fl;
    for (; k + 7 * SF < F; k += 8 * SF) {
      block4(k);
      block4(k + 4 * SF);
    }
    if (k + 3 * SF < F) {
      block4(k);
      k += 4 * SF;
    }
    if (k < F) {   // the last one to three points
      double pb[NB], R[NB];
#pragma unroll
      for (int cI = 0; cI < NB; ++cI) pb[cI] = 0.0;
      for (; k < F; k += SF) {
        const double wr = resid(ld(om, k), ld(epi, k), R);
#pragma unroll
        for (int cI = 0; cI < NB; ++cI) pb[cI] = __builtin_fma(R[cI], wr, pb[cI]);
      }
#pragma unroll
      for (int cI = 0; cI < NB; ++cI) kahan_fma_acc(gv[cI], gl[cI], 1.0, pb[cI]);
    }
    {
      double ngl[NB];
#pragma unroll
      for (int cI = 0; cI < NB; ++cI) ngl[cI] = -gl[cI];
      freq_sum_dd_n<NB>(gv, ngl, SP, SL);
    }
    if constexpr (GRAD) freq_sum_n<NB>(Sv, SP, SL);
#pragma unroll
    for (int cI = 0; cI < NB; ++cI) {
      gv[cI] = gv[cI] * ts[cI];
      if constexpr (GRAD) Sv[cI] = Sv[cI] * pole_scale<NB>(sq, cI);
    }
  }

  // correction: zt += A^-1 (D^-1 g - damping zt)
  if (refine) {
    if constexpr (SP == 1) {
      double dz[N];
#pragma unroll
      for (int i = 0; i < N; ++i) dz[i] = __builtin_fma(gv[i], invd_r[i], -damping * zt[i]);
      double Af[S::NT], uf[N];
      unpark<N>(lds_all, WAVE / SL, grp, Af, uf);
      chol_solve<N>(Af, uf, dz);
#pragma unroll
      for (int i = 0; i < N; ++i) zt[i] += dz[i];
    } else {
      const LdsLayout<N> lay(L);
      double *A = lay.A, *uinv = lay.uinv, *vw = lay.vw;
#pragma unroll
      for (int cI = 0; cI < NB; ++cI) {
        const int p = q * NB + cI;
        if (p < N) vw[p] = __builtin_fma(gv[cI], invd_own[cI], -damping * zt[cI]);
      }
      __syncthreads();
      lds_chol_solve<N>((lds_cptr)A, (lds_cptr)uinv, (lds_ptr)vw);
      __syncthreads();
#pragma unroll
      for (int cI = 0; cI < NB; ++cI) {
        const int p = q * NB + cI;
        zt[cI] += p < N ? vw[p] : 0.0;
      }
    }
  }
  double wv_[NB];
  double ws_part = 0.0;
#pragma unroll
  for (int cI = 0; cI < NB; ++cI) {
    zc[cI] = zt[cI] * invd_own[cI];
    wv_[cI] = flip ? fabs(zc[cI]) : zc[cI];
    if constexpr (GRAD) ws_part = __builtin_fma(wv_[cI], Sv[cI], ws_part);
  }
  // eps_inf: the adjoint takes it from the column sums before its pass 3.
  // The forward kernels take it from the cost pass: with v_k = eps'_k -
  // (R w)_k, eps_inf is the mean of v and the real part of the cost is
  // sum (v - mean)^2 = sum (v - K)^2 - (sum (v - K))^2 / F for any shift K.
  // K = v_0 (the first point) differs from the mean by about one residual,
  // so the subtraction loses at most a few digits of the cost's last bits.
  double einf = 0.0, shift = 0.0;
  if constexpr (GRAD) {
    einf = (F > 0) ? (sum_er - group_sum<SP>(ws_part)) / (double)F : 0.0;
    shift = einf;
  } else if (F > 0) {
    const double w0 = ld(om, 0);
    double Rv[NB];
    basis_Rs<NB>(w0 * w0, tau2s, sq, Rv);
    double pr = 0.0;
#pragma unroll
    for (int cI = 0; cI < NB; ++cI) pr = __builtin_fma(wv_[cI] * pole_scale<NB>(sq, cI), Rv[cI], pr);
    shift = ld(epr, 0) - group_sum<SP>(pr);
  }

  // ---- pass 3: residuals and cost (+ g_w for the adjoint)
  double gw[GRAD ? NB : 1], gw2[GRAD ? NB : 1], wt[NB];
#pragma unroll
  for (int cI = 0; cI < (GRAD ? NB : 1); ++cI) gw[cI] = gw2[cI] = 0.0;
#pragma unroll
  for (int cI = 0; cI < NB; ++cI) wt[cI] = wv_[cI] * tau_of(cI);
  // from the basis values of every point (grouped form: the weights carry the
  // scales, and the adjoint's sums g_w get theirs afterwards); rr is
  // eps' - shift - R w, and sa collects its sum (the forward kernels' shifted
  // mean)
  auto pass3_basis = [&](double &sa) -> double {
    double acc = 0.0;
    double wvs[NB], wts[NB];
#pragma unroll
    for (int cI = 0; cI < NB; ++cI) {
      wvs[cI] = wv_[cI] * pole_scale<NB>(sq, cI);
      wts[cI] = wv_[cI] * ts[cI];
    }
    sa = 0.0;
    int64_t k = fl;
    double w_n = 0, er_n = 0, ei_n = 0;
    if (k < F) {
      w_n = ld_first(om, k);
      er_n = ld_first(epr, k);
      ei_n = ld_first(epi, k);
    }
    for (; k < F; k += SF) {
      const double w = w_n, er = er_n, ei = ei_n;
      const int64_t kn = (k + SF < F) ? k + SF : k;   // in-bounds prefetch, no branch
      w_n = ld(om, kn);
      er_n = ld(epr, kn);
      ei_n = ld(epi, kn);
      double Rv[NB];
      basis_Rs<NB>(w * w, tau2s, sq, Rv);
      double pr = 0.0, pi = 0.0;
#pragma unroll
      for (int cI = 0; cI < NB; ++cI) {
        pr = __builtin_fma(wvs[cI], Rv[cI], pr);
        pi = __builtin_fma(wts[cI], Rv[cI], pi);
      }
      const double rr = (er - shift) - group_sum<SP>(pr);
      const double ri = __builtin_fma(-w, group_sum<SP>(pi), ei);
      if constexpr (!GRAD) sa += rr;
      acc = __builtin_fma(rr, rr, acc);
      acc = __builtin_fma(ri, ri, acc);
      if constexpr (GRAD) {
        // g_w = R^T r' + I^T r'' = s ((R/s)^T r' + tau ((R/s)^T (w r'')))
        const double wri = w * ri;
#pragma unroll
        for (int cI = 0; cI < NB; ++cI) {
          gw[cI] = __builtin_fma(Rv[cI], rr, gw[cI]);
          gw2[cI] = __builtin_fma(Rv[cI], wri, gw2[cI]);
        }
      }
    }
    return acc;
  };
  double cost, sa = 0.0;
  // lanes whose partial sums are added at the end: the frequency lanes of the
  // pole group (basis form: the pole group's sums are combined per point), or
  // all lanes of the candidate (rational form over the whole candidate)
  int red_from = SP;
  if constexpr (GRAD) {
    cost = pass3_basis(sa);
  } else {
    // (lanes whose cost is replaced by their status do not count)
    const bool matters = active && !bad && ok;
    bool use_basis = !flip;
    if (!use_basis) {
      if constexpr (SP == 1) {
        double tau2v[NB];
#pragma unroll
        for (int cI = 0; cI < NB; ++cI) tau2v[cI] = tau2_of(cI);
        use_basis = rational_cost_pass<NB, 1>(tau2v, wv_, wt, matters, fl, SF, F, om, epr, epi, shift, ld, ld_first,
                                             cost, sa);
      } else {
        // every lane of the candidate takes all N poles (gathered through the
        // candidate's LDS region, whose right-hand-side, first-solution and
        // scaling vectors are free after the solves) and every SL-th point:
        // one rational function of degree N per point instead of SP of degree
        // NB combined across lanes
        const LdsLayout<N> lay(L);
        double *t2s = lay.vb, *wsh = lay.vz, *wts = lay.invd;
        __syncthreads();
#pragma unroll
        for (int cI = 0; cI < NB; ++cI) {
          const int p = q * NB + cI;
          if (p < N) {
            t2s[p] = tau2_of(cI);
            wsh[p] = wv_[cI];
            wts[p] = wt[cI];
          }
        }
        __syncthreads();
        use_basis = rational_cost_pass<N, 1>(t2s, wsh, wts, matters, sub, SL, F, om, epr, epi, shift, ld, ld_first,
                                            cost, sa);
        red_from = 1;
      }
    }
    if (use_basis) {
      cost = pass3_basis(sa);
      red_from = SP;
    }
  }
  cost = freq_sum(cost, red_from, SL);
  if constexpr (!GRAD) {
    sa = freq_sum(sa, red_from, SL);
    if (F > 0) {
      cost -= sa * (sa / (double)F);
      einf = shift + sa / (double)F;
    }
  }

  const bool sing = !ok;
  const int st = bad ? ST_BADINPUT : (sing ? ST_SINGULAR : ST_OK);
  const bool writer = active && fl == 0;
  double gc = 1.0;
  if (writer && q == 0) {
    a.cost[c] = st == ST_OK ? cost : (st == ST_SINGULAR ? INFINITY : NAN);
    if (a.eps_inf) a.eps_inf[c] = st == ST_OK ? einf : NAN;
    if (a.status) a.status[c] = (int8_t)st;
  }
  if (writer && a.weights) {
#pragma unroll
    for (int cI = 0; cI < NB; ++cI) {
      const int p = q * NB + cI;
      if (p < N) a.weights[c * a.ld + p] = st == ST_OK ? wv_[cI] : NAN;
    }
  }
  if constexpr (!GRAD) {
    return;
  } else {
    // ---- adjoint: mu = M^-1 (s o g_w), M = D A D
    if (a.grad_cost) gc = active ? a.grad_cost[c] : 0.0;
    double mt[NB], mu[NB];
    freq_sum_n<NB>(gw2, SP, SL);
    freq_sum_n<NB>(gw, SP, SL);
#pragma unroll
    for (int cI = 0; cI < NB; ++cI) {
      gw[cI] = -2.0 * pole_scale<NB>(sq, cI) * __builtin_fma(tau_of(cI), gw2[cI], gw[cI]);
      const double s = (flip && zc[cI] < 0.0) ? -1.0 : 1.0;
      mt[cI] = s * gw[cI] * invd_own[cI];
    }
    if constexpr (SP == 1) {
      double Af[S::NT], uf[N];
      unpark<N>(lds_all, WAVE / SL, grp, Af, uf);
      chol_solve<N>(Af, uf, mt);
    } else {
      const LdsLayout<N> lay(L);
      double *A = lay.A, *uinv = lay.uinv, *vw = lay.vw;
#pragma unroll
      for (int cI = 0; cI < NB; ++cI) {
        const int p = q * NB + cI;
        if (p < N) vw[p] = mt[cI];
      }
      __syncthreads();
      lds_chol_solve<N>((lds_cptr)A, (lds_cptr)uinv, (lds_ptr)vw);
      __syncthreads();
#pragma unroll
      for (int cI = 0; cI < NB; ++cI) {
        const int p = q * NB + cI;
        mt[cI] = p < N ? vw[p] : 0.0;
      }
    }
#pragma unroll
    for (int cI = 0; cI < NB; ++cI) mu[cI] = mt[cI] * invd_own[cI];

    // ---- pass 4: basis derivatives against the residuals.  With x^2 R = 1 - R,
    // dR/dtheta = -2 ln10 I^2 and dI/dtheta = ln10 I (2R - 1); ln10 is applied
    // after the sums, and the dot products run over R with tau-scaled weights
    // as in the forward passes.
    double T1[NB], T2[NB], T3[NB], T4[NB], zt4[NB], mt4[NB], tv4[NB], tv4s[NB];
#pragma unroll
    for (int cI = 0; cI < NB; ++cI) {
      T1[cI] = T2[cI] = T3[cI] = T4[cI] = 0.0;
      tv4[cI] = tau_of(cI);
      tv4s[cI] = tau2_of(cI);
      zt4[cI] = zc[cI] * tv4[cI];
      mt4[cI] = mu[cI] * tv4[cI];
    }
    {
      int64_t k = fl;
      double w_n = 0, er_n = 0, ei_n = 0;
      if (k < F) {
        w_n = ld_first(om, k);
        er_n = ld_first(epr, k);
        ei_n = ld_first(epi, k);
      }
      for (; k < F; k += SF) {
        const double w = w_n, er = er_n, ei = ei_n;
        const int64_t kn = (k + SF < F) ? k + SF : k;
        w_n = ld(om, kn);
        er_n = ld(epr, kn);
        ei_n = ld(epi, kn);
        double Rv[NB];
        basis_R<NB>(w * w, tv4s, Rv);
        double pr = 0.0, pi = 0.0, pz = 0.0, pm = 0.0;
#pragma unroll
        for (int cI = 0; cI < NB; ++cI) {
          pr = __builtin_fma(wv_[cI], Rv[cI], pr);
          pi = __builtin_fma(wt[cI], Rv[cI], pi);
          pz = __builtin_fma(zt4[cI], Rv[cI], pz);
          pm = __builtin_fma(mt4[cI], Rv[cI], pm);
        }
        const double rr = (er - einf) - group_sum<SP>(pr);
        const double ri = __builtin_fma(-w, group_sum<SP>(pi), ei);
        const double qz = __builtin_fma(-w, group_sum<SP>(pz), ei);
        const double qm = w * group_sum<SP>(pm);
        const double m2rr = -2.0 * rr;
#pragma unroll
        for (int cI = 0; cI < NB; ++cI) {
          const double R = Rv[cI];
          const double I = (w * tv4[cI]) * R;
          const double dI = I * __builtin_fma(2.0, R, -1.0);
          T1[cI] = __builtin_fma(I * m2rr, I, __builtin_fma(dI, ri, T1[cI]));
          T2[cI] = __builtin_fma(dI, qz, T2[cI]);
          T3[cI] = __builtin_fma(dI, qm, T3[cI]);
          T4[cI] = __builtin_fma(dI, I, T4[cI]);
        }
      }
    }
    freq_sum_n<NB>(T1, SP, SL);
    freq_sum_n<NB>(T2, SP, SL);
    freq_sum_n<NB>(T3, SP, SL);
    freq_sum_n<NB>(T4, SP, SL);
#pragma unroll
    for (int cI = 0; cI < NB; ++cI) {
      T1[cI] = LN10 * T1[cI];
      T2[cI] = LN10 * T2[cI];
      T3[cI] = LN10 * T3[cI];
      T4[cI] = LN10 * T4[cI];
    }
    if (writer) {
      // padding entries of the row (poles beyond this material's count) are 0
      if (q == 0 && a.grad_theta)
        for (int64_t p = N; p < a.ld; ++p) a.grad_theta[c * a.ld + p] = 0.0;
#pragma unroll
      for (int cI = 0; cI < NB; ++cI) {
        const int p = q * NB + cI;
        if (p >= N) continue;
        double g = -2.0 * wv_[cI] * T1[cI] + mu[cI] * T2[cI] - zc[cI] * T3[cI] -
                   2.0 * damping * mu[cI] * zc[cI] * T4[cI];
        if (a.grad_theta) a.grad_theta[c * a.ld + p] = st == ST_OK ? gc * g : NAN;
        // per-candidate record for the target gradient: [w | z | mu | tau | eps_inf, gc]
        if (a.record) {
          double *rec = a.record + c * a.rec_ld;
          rec[p] = wv_[cI];
          rec[N + p] = zc[cI];
          rec[2 * N + p] = mu[cI];
          rec[3 * N + p] = tv4[cI];
          if (p == 0) {
            rec[4 * N] = einf;
            rec[4 * N + 1] = st == ST_OK ? gc : 0.0;
          }
        }
      }
    }
  }
}

// The cost kernel: one tile per 64-lane block.  XCD-aware tile order:
// workgroups are dealt round-robin to the 8 XCDs, so block b runs on XCD
// b % 8 as its (b / 8)-th block.  The plan gives every XCD its own list of
// tiles (whole materials where possible, so that a material's spectra stay in
// one L2; the lists balanced by work, each longest first).  The grid covers
// the longest list; surplus blocks exit.
template <int N, int SP, bool GRAD, int UNI>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(waves_per_simd<N, SP, GRAD, UNI>())))
void fit_kernel(const FitArgs a) {
  const int xcd = blockIdx.x & 7;
  const int64_t j = blockIdx.x >> 3;
  if (j >= a.xcd_off[xcd + 1] - a.xcd_off[xcd]) return;
  fit_tile<N, SP, GRAD, UNI>(a, a.xcd_off[xcd] + j);
}

// The forward kernel with the refinement pass in double-double, general tiles.
template <int N, int SP>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(waves_per_simd<N, SP, false, 0>())))
void fit_dd_kernel(const FitArgs a) {
  const int xcd = blockIdx.x & 7;
  const int64_t j = blockIdx.x >> 3;
  if (j >= a.xcd_off[xcd + 1] - a.xcd_off[xcd]) return;
  fit_tile<N, SP, false, 0, true>(a, a.xcd_off[xcd] + j);
}

// Pole split by pole count, measured per bucket on the ragged workload (each
// pole count alone, autotuned frequency split): one lane per candidate up to
// N = 11 (at N = 9..11 its register spills cost less than the DPP traffic and
// the padded pole of the two-lane ring; at N = 12 they do not), two lanes up
// to N = 16 (N = 13..16 pad to 16 on four lanes), four above (two lanes
// spill the adjoint heavily at N = 17, 18).
constexpr int pole_split_for(int n) { return n <= 11 ? 1 : (n <= 16 ? 2 : 4); }

// Blocks of a cost-kernel grid: eight times the longest of the 8 XCD tile
// lists (block b runs tile b / 8 of XCD b % 8's list).
inline unsigned fit_grid_blocks(const FitArgs &a) {
  int64_t longest = 0;
  for (int x = 0; x < 8; ++x) longest = a.xcd_off[x + 1] - a.xcd_off[x] > longest ? a.xcd_off[x + 1] - a.xcd_off[x] : longest;
  return (unsigned)(longest * 8);
}

// Launch of the cost kernel for N poles: the adjoint (GRAD) or the forward
// kernel, in the uniform-tile form the plan found (split 1: scalar spectrum
// loads; wider splits: per-lane offsets) or the general one.  The grid covers
// the longest of the 8 XCD tile lists.
template <int N, bool GRAD> hipError_t launch_fit_variant(const FitArgs &a, int64_t n_tiles, bool uni, hipStream_t s) {
  constexpr int SP = pole_split_for(N);
  const size_t lds = (size_t)Shape<N, SP>::LDS_DOUBLES * 8 * a.cand_per_wave;
  FitArgs b = a;
  b.n_tiles = n_tiles;
  const unsigned blocks = fit_grid_blocks(a);
  if (blocks == 0) return hipSuccess;
  if (uni && a.freq_split == 1)
    hipLaunchKernelGGL((fit_kernel<N, SP, GRAD, 1>), dim3(blocks), dim3(64), lds, s, b);
  else if (uni)
    hipLaunchKernelGGL((fit_kernel<N, SP, GRAD, 2>), dim3(blocks), dim3(64), lds, s, b);
  else
    hipLaunchKernelGGL((fit_kernel<N, SP, GRAD, 0>), dim3(blocks), dim3(64), lds, s, b);
  return hipGetLastError();
}

// The forward kernel with the extended-precision refinement: the general
// tile form only (it serves uniform tiles too).
template <int N> hipError_t launch_fit_dd_variant(const FitArgs &a, int64_t n_tiles, hipStream_t s) {
  constexpr int SP = pole_split_for(N);
  const size_t lds = (size_t)Shape<N, SP>::LDS_DOUBLES * 8 * a.cand_per_wave;
  FitArgs b = a;
  b.n_tiles = n_tiles;
  const unsigned blocks = fit_grid_blocks(a);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((fit_dd_kernel<N, SP>), dim3(blocks), dim3(64), lds, s, b);
  return hipGetLastError();
}

}  // namespace dfit
