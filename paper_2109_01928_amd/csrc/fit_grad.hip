// Adjoint instantiations of the cost kernel (fit_kernel.hpp with GRAD), in a
// translation unit of their own so that they compile beside the forward ones.

#include "fit_kernel.hpp"

namespace dfit {

namespace {
template <int... Ns> struct GradTable {
  static hipError_t fit(int n, const FitArgs &a, int64_t tiles, bool uni, hipStream_t s) {
    hipError_t e = hipErrorInvalidValue;
    ((n == Ns ? (e = launch_fit_variant<Ns, true>(a, tiles, uni, s)) : hipSuccess), ...);
    return e;
  }
};
}  // namespace

hipError_t launch_fit_grad(int n, const FitArgs &a, int64_t n_tiles, bool uni, hipStream_t s) {
  return GradTable<1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24>::fit(
      n, a, n_tiles, uni, s);
}

}  // namespace dfit
