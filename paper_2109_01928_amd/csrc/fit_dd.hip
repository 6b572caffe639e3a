// Forward cost kernels with the refinement pass in double-double
// (FLAG_DD_REFINE), in a translation unit of their own so that they compile
// beside the others.

#include "fit_kernel.hpp"

namespace dfit {

namespace {
template <int... Ns> struct DdTable {
  static hipError_t fit(int n, const FitArgs &a, int64_t tiles, hipStream_t s) {
    hipError_t e = hipErrorInvalidValue;
    ((n == Ns ? (e = launch_fit_dd_variant<Ns>(a, tiles, s)) : hipSuccess), ...);
    return e;
  }
};
}  // namespace

hipError_t launch_fit_dd(int n, const FitArgs &a, int64_t n_tiles, hipStream_t s) {
  return DdTable<1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24>::fit(
      n, a, n_tiles, s);
}

}  // namespace dfit
