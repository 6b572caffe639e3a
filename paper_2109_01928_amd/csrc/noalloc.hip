// debye_fit_eval_grad_noalloc: the cost, its adjoint and the target
// gradients without any device allocation, for callers that cannot allocate.
// The per-candidate adjoint records that the target-gradient kernel reads
// back live in `scratch`, a file-scope device array of fixed size: every GPU
// the library runs on holds its own copy of it for the life of the process,
// and every call on that GPU shares it (calls that overlap on one GPU race).

#include <cstdio>
#include <map>
#include <mutex>

#include "../../include/debyefit.h"
#include "common.hpp"
#include "fit_eval.hpp"

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;   // 64 MiB per GPU

// In host code `scratch` only names the symbol: its device address comes
// from hipGetSymbolAddress, once per device, and only that address is used.
__device__ __align__(256) double scratch[SCRATCH_BYTES / sizeof(double)];

std::mutex g_mutex;
std::map<int, double *> g_ptr;   // device ordinal -> device address of its `scratch`

// the records' buffer: this device's `scratch`, if it is large enough
int scratch_records(size_t bytes, double **out) {
  if (bytes > SCRATCH_BYTES) {
    char msg[256];
    snprintf(msg, sizeof msg,
             "debye_fit_eval_grad_noalloc: the adjoint records need %zu bytes, more than the %zu-byte static "
             "workspace (use debye_fit_eval_grad with a DEBYE_PLAN_TARGET_GRAD plan)",
             bytes, SCRATCH_BYTES);
    return dfit::set_error(DEBYE_ERANGE, msg);
  }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return dfit::set_error(DEBYE_EHIP, hipGetErrorString(e));
  std::lock_guard<std::mutex> lock(g_mutex);
  auto it = g_ptr.find(dev);
  if (it == g_ptr.end()) {
    // first use on this device (it is the current one): its copy's address
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return dfit::set_error(DEBYE_EHIP, "hipGetSymbolAddress(scratch) failed");
    it = g_ptr.emplace(dev, (double *)ptr).first;
  }
  *out = it->second;
  return DEBYE_OK;
}

}  // namespace

extern "C" int debye_fit_eval_grad_noalloc(const debye_plan *plan, const debye_batch *b, const double *log10_tau,
                                           int64_t ld, double damping, uint32_t flags, const double *grad_cost,
                                           double *cost, double *grad_log10_tau, double *grad_eps_re,
                                           double *grad_eps_im, int8_t *status, hipStream_t stream) {
  return dfit::fit_eval_grad_external(plan, b, log10_tau, ld, damping, flags, grad_cost, cost, grad_log10_tau,
                                      grad_eps_re, grad_eps_im, status, scratch_records, stream);
}
