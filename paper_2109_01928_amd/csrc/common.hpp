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
enum { FLAG_NO_SIGN_FLIP = 1u };

// Reciprocal of d >= 1.  The hardware estimate r0 has a relative error e
// below 2^-24; one third-order Newton-Raphson step (Householder's iteration
// for 1/d) r = r0 (1 + e + e^2), e = 1 - d r0, leaves an error of order e^3
// (about 2^-72) before the final rounding, so the result is within half an
// ulp of 1/d (measured on 2^20 inputs in [1, 1e12]).
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

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// multiply/xor bijection on four 64-bit words with a Weyl-sequence key.
// ---------------------------------------------------------------------------
struct U64x4 {
  uint64_t w[4];
};

__device__ __forceinline__ U64x4 philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                             uint64_t k1) {
  const uint64_t mA = 0xD2E7470EE14C6C93ULL, mB = 0xCA5A826395121157ULL;
  const uint64_t wA = 0x9E3779B97F4A7C15ULL, wB = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t hA = __umul64hi(mA, c0), lA = mA * c0;
    const uint64_t hB = __umul64hi(mB, c2), lB = mB * c2;
    const uint64_t n0 = hB ^ c1 ^ k0, n2 = hA ^ c3 ^ k1;
    c0 = n0;
    c1 = lB;
    c2 = n2;
    c3 = lA;
    k0 += wA;
    k1 += wB;
  }
  U64x4 r;
  r.w[0] = c0;
  r.w[1] = c1;
  r.w[2] = c2;
  r.w[3] = c3;
  return r;
}

// top 53 bits as a double in [0, 1)
__device__ __forceinline__ double unit53(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

enum { STREAM_PSO_INIT = 0, STREAM_PSO_STEP = 1, STREAM_NOISE = 2, STREAM_DE_INIT = 3, STREAM_DE_TRIAL = 4,
       STREAM_DE_CROSS = 5, STREAM_DE_F = 6, STREAM_DA_INIT = 7, STREAM_DA_VISIT = 8, STREAM_DA_ACCEPT = 9 };

}  // namespace dfit
