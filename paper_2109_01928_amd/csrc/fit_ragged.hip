// One persistent launch for a whole ragged evaluation: every pole-count
// bucket of a plan in a single kernel.  The plan lists work items (bucket,
// tile) per XCD, longest first by estimated duration across all buckets;
// each block (one wavefront) takes the next item of its XCD's list through a
// counter in device memory (a vector atomic from one lane) until the list is
// exhausted, and runs the cost-kernel body of that bucket's pole count on the
// tile.  Blocks are dealt round-robin to the XCDs, so block b serves XCD b % 8
// and a material's spectra stay in that XCD's L2.

#include "fit_kernel.hpp"

namespace dfit {

namespace {

// variant of the body a bucket runs: pole count and tile form (uniform tiles
// with a wave-uniform spectrum base, or general)
template <int N> __device__ __forceinline__ void ragged_tile(const FitArgs &a, int64_t tile, bool uni) {
  constexpr int SP = pole_split_for(N);
  if (uni) fit_tile<N, SP, false, 2>(a, tile);
  else fit_tile<N, SP, false, 0>(a, tile);
}

template <int... Ns> struct RaggedSwitch {
  __device__ __forceinline__ static void run(int n, const FitArgs &a, int64_t tile, bool uni) {
    ((n == Ns ? (ragged_tile<Ns>(a, tile, uni), 0) : 0), ...);
  }
};

}  // namespace

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void fit_ragged_kernel(const RaggedArgs r) {
  const int xcd = blockIdx.x & 7;
  const int64_t first = r.item_off[xcd], n_items = r.item_off[xcd + 1] - first;
  for (;;) {
    int32_t next = 0;
    if (threadIdx.x == 0) next = atomicAdd(&r.counters[xcd], 1);
    next = __builtin_amdgcn_readfirstlane(next);
    if (next >= n_items) break;
    const int64_t item = r.items[first + next];
    const int32_t b = __builtin_amdgcn_readfirstlane((int32_t)(item >> 40));
    const int64_t tile = item & (((int64_t)1 << 40) - 1);
    const RaggedBucket bk = r.buckets[b];
    FitArgs a = r.common;
    a.freq_split = bk.freq_split;
    a.cand_per_wave = bk.cand_per_wave;
    a.lane_cand = bk.lane_cand;
    a.lane_mat = bk.lane_mat;
    RaggedSwitch<1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24>::run(
        bk.n_poles, a, tile, bk.uni != 0);
  }
}

// counters back to 0 (a kernel, so that the evaluation can be captured)
__global__ void ragged_reset_kernel(int32_t *counters) {
  if (threadIdx.x < 8) counters[threadIdx.x] = 0;
}

hipError_t launch_fit_ragged(const RaggedArgs &r, int32_t blocks, size_t lds_bytes, hipStream_t s) {
  hipLaunchKernelGGL(ragged_reset_kernel, dim3(1), dim3(64), 0, s, r.counters);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fit_ragged_kernel, dim3((unsigned)blocks), dim3(64), lds_bytes, s, r);
  return hipGetLastError();
}

}  // namespace dfit
