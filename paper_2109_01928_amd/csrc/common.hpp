// Device helpers shared by the gfx950 kernels of the Debye fitting library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dfit {

constexpr int WAVE = 64;
#define DFIT_MAX_POLES 24
#define DFIT_MAX_MEM 32
constexpr double LN10 = 2.302585092994045684017991454684364208;
constexpr double THETA_LIMIT = 30.0;  // |log10 tau| beyond this is rejected (status BADINPUT)

enum { ST_OK = 0, ST_BADINPUT = 1, ST_SINGULAR = 2 };
enum { FLAG_NO_SIGN_FLIP = 1u, FLAG_NO_REFINE = 2u, FLAG_DD_REFINE = 4u };

// Reciprocal of a d whose reciprocal is a normal number (the callers pass d
// in [2^-1012, 2^990]).  The hardware estimate r0 has a relative error e
// below 2^-24; one third-order Newton-Raphson step (Householder's iteration
// for 1/d) r = r0 (1 + e + e^2), e = 1 - d r0, leaves an error of order e^3
// (about 2^-72) before the final rounding, so the result is within half an
// ulp of 1/d (measured on 2^20 log-uniform inputs in [1, 1e12] and in
// [2^-1012, 2^990]).
__device__ __forceinline__ double rcp_nr(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  const double e = __builtin_fma(-d, r, 1.0);
  return __builtin_fma(r, __builtin_fma(e, e, e), r);
}

// Cross-lane move of a double inside a quad (DPP quad_perm; CTRL encodes the
// source lane of each of the four lanes, two bits per lane).
// Every source lane of a quad permutation is valid, so the move needs no
// "old" value (bound_ctrl set) and compiles to two bare v_mov_b32_dpp.
template <int CTRL> __device__ __forceinline__ double dpp_quad(double v) {
  int lo = __builtin_amdgcn_mov_dpp((int)__double2loint(v), CTRL, 0xF, 0xF, true);
  int hi = __builtin_amdgcn_mov_dpp((int)__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
constexpr int QP_SWAP1 = 0xB1;  // [1,0,3,2]: lane ^ 1
constexpr int QP_ROT1 = 0x39;   // [1,2,3,0]: (lane + 1) mod 4
constexpr int QP_SWAP2 = 0x4E;  // [2,3,0,1]: lane ^ 2 = (lane + 2) mod 4

}  // namespace dfit
