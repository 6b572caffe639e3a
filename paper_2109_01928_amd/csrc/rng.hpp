// Counter-based random numbers of the optimisers and the table noise.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dfit {

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
