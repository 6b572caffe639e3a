// Automatic number of Debye poles (paper Sec. III-B): fit with 1, 2, ...
// poles until the average fractional error is below the target or the
// maximum pole count is reached.  Host orchestration of the library's own
// entry points: every round fits the unresolved materials with the next
// `chunk` pole counts as one ragged batch (swarm, polish, weights, error).

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/debyefit.h"
#include "common.hpp"
#include "fit_eval.hpp"

namespace {

struct DevBuf {
  void *p = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  bool alloc(size_t bytes) {
    if (p) (void)hipFree(p);
    p = nullptr;
    return hipMalloc(&p, bytes ? bytes : 8) == hipSuccess;
  }
  template <class T> T *as() const { return (T *)p; }
};

struct PlanHolder {
  debye_plan *p = nullptr;
  ~PlanHolder() {
    if (p) debye_plan_destroy(p);
  }
};

int hip_err(hipError_t e, const char *what) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
  return dfit::set_error(DEBYE_EHIP, buf);
}

#define AUTO_HIP(expr, what)                   \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return hip_err(e_, what); \
  } while (0)

template <class T> int upload(DevBuf &d, const std::vector<T> &h, hipStream_t s) {
  if (!d.alloc(h.size() * sizeof(T))) return dfit::set_error(DEBYE_ENOMEM, "automatic poles: allocation failed");
  if (!h.empty()) AUTO_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s), "upload");
  return DEBYE_OK;
}

int alloc_doubles(DevBuf &d, size_t n) {
  return d.alloc(n * 8) ? DEBYE_OK : dfit::set_error(DEBYE_ENOMEM, "automatic poles: allocation failed");
}

}  // namespace

extern "C" int debye_fit_auto(const debye_batch *mats, const int64_t *f_off_host, const double *lb, const double *ub,
                              debye_auto_params p, double damping, uint32_t flags, int32_t *n_poles_out,
                              double *log10_tau_out, double *weights_out, double *eps_inf_out, double *afe_out,
                              int64_t ld_out, hipStream_t stream) {
  using dfit::set_error;
  if (!mats || !f_off_host || !lb || !ub || !n_poles_out || !log10_tau_out || !weights_out || !eps_inf_out ||
      !afe_out)
    return set_error(DEBYE_EINVAL, "automatic poles: NULL pointer");
  if (!mats->f_off || !mats->omega || !mats->eps_re || !mats->eps_im)
    return set_error(DEBYE_EINVAL, "automatic poles: batch has a NULL spectra pointer");
  const int32_t M = mats->n_mat;
  if (M < 1) return set_error(DEBYE_ERANGE, "automatic poles: n_mat must be >= 1");
  if (p.n_min < 1 || p.n_max < p.n_min || p.n_max > DEBYE_MAX_POLES || p.chunk < 1 || p.particles < 1 ||
      p.iters < 0 || p.polish_steps < 0 || !(p.afe_target > 0.0))
    return set_error(DEBYE_ERANGE, "automatic poles: parameters out of range");
  if (ld_out < p.n_max) return set_error(DEBYE_ERANGE, "automatic poles: ld_out < n_max");
  if (f_off_host[0] != 0 || f_off_host[M] != mats->n_freq)
    return set_error(DEBYE_EINVAL, "automatic poles: f_off does not match n_freq");
  for (int32_t m = 0; m < M; ++m)
    if (f_off_host[m + 1] - f_off_host[m] < 1) return set_error(DEBYE_ERANGE, "automatic poles: empty spectrum");

  std::vector<double> lb_h(M), ub_h(M);
  AUTO_HIP(hipMemcpyAsync(lb_h.data(), lb, (size_t)M * 8, hipMemcpyDeviceToHost, stream), "bounds");
  AUTO_HIP(hipMemcpyAsync(ub_h.data(), ub, (size_t)M * 8, hipMemcpyDeviceToHost, stream), "bounds");
  AUTO_HIP(hipStreamSynchronize(stream), "sync");

  std::vector<int32_t> final_n(M, 0);
  std::vector<double> final_einf(M, NAN), final_afe(M, NAN);
  std::vector<int32_t> unresolved(M);
  for (int32_t m = 0; m < M; ++m) unresolved[m] = m;
  const int64_t P = p.particles;

  // Entry e = m * NN + (N - n_min) for every (material, pole count): its swarm
  // uses Philox key (seed, e) whatever the round and the chunk, so the fit of
  // (m, N) does not depend on how the sweep is cut.  Entries outside the
  // round carry no particles and one copied frequency point.
  const int32_t NN = p.n_max - p.n_min + 1;
  const int64_t E = (int64_t)M * NN;
  std::vector<char> in_round(M);
  for (int32_t n0 = p.n_min; n0 <= p.n_max && !unresolved.empty(); n0 += p.chunk) {
    const int32_t n1 = std::min(p.n_max, n0 + p.chunk - 1);
    const int32_t K = n1 - n0 + 1;
    const int32_t ld = n1;
    std::fill(in_round.begin(), in_round.end(), 0);
    for (int32_t m : unresolved) in_round[m] = 1;
    std::vector<int32_t> src_mat(E), n_e(E);
    std::vector<int64_t> f_e(E + 1), c_e(E + 1), one(E + 1);
    std::vector<double> lb_e(E), ub_e(E);
    f_e[0] = c_e[0] = 0;
    for (int64_t e = 0; e < E; ++e) {
      const int32_t m = (int32_t)(e / NN), N = p.n_min + (int32_t)(e % NN);
      const bool active = in_round[m] && N >= n0 && N <= n1;
      src_mat[e] = m;
      n_e[e] = active ? N : n0;
      f_e[e + 1] = f_e[e] + (active ? f_off_host[m + 1] - f_off_host[m] : 1);
      c_e[e + 1] = c_e[e] + (active ? P : 0);
      lb_e[e] = lb_h[m];
      ub_e[e] = ub_h[m];
      one[e] = e;
    }
    one[E] = E;
    const int64_t FE = f_e[E], PE = c_e[E];
    DevBuf d_src, d_n, d_f, d_c, d_one, d_lb, d_ub, d_om, d_er, d_ei;
    int rc;
    if ((rc = upload(d_src, src_mat, stream)) || (rc = upload(d_n, n_e, stream)) || (rc = upload(d_f, f_e, stream)) ||
        (rc = upload(d_c, c_e, stream)) || (rc = upload(d_one, one, stream)) || (rc = upload(d_lb, lb_e, stream)) ||
        (rc = upload(d_ub, ub_e, stream)) || (rc = alloc_doubles(d_om, FE)) || (rc = alloc_doubles(d_er, FE)) ||
        (rc = alloc_doubles(d_ei, FE)))
      return rc;
    AUTO_HIP(dfit::launch_gather_spectra(E, mats->f_off, d_src.as<int32_t>(), d_f.as<int64_t>(), mats->omega,
                                         mats->eps_re, mats->eps_im, d_om.as<double>(), d_er.as<double>(),
                                         d_ei.as<double>(), stream),
             "gather spectra");
    debye_batch be{};
    be.n_mat = (int32_t)E;
    be.max_poles = n1;
    be.n_freq = FE;
    be.n_cand = PE;
    be.f_off = d_f.as<int64_t>();
    be.cand_off = d_c.as<int64_t>();
    be.n_poles = d_n.as<int32_t>();
    be.omega = d_om.as<double>();
    be.eps_re = d_er.as<double>();
    be.eps_im = d_ei.as<double>();
    debye_batch b1 = be;
    b1.n_cand = E;
    b1.cand_off = d_one.as<int64_t>();

    // swarms
    DevBuf x, v, pbx, pbc, gbx, gbc, gbi, cost;
    if ((rc = alloc_doubles(x, PE * ld)) || (rc = alloc_doubles(v, PE * ld)) || (rc = alloc_doubles(pbx, PE * ld)) ||
        (rc = alloc_doubles(pbc, PE)) || (rc = alloc_doubles(gbx, E * ld)) || (rc = alloc_doubles(gbc, E)) ||
        (rc = alloc_doubles(gbi, E)) || (rc = alloc_doubles(cost, PE)))
      return rc;
    // entries outside the round keep a valid (unused) best for the polish below
    AUTO_HIP(dfit::launch_fill(gbx.as<double>(), E * ld, 0.0, stream), "fill");
    PlanHolder plan;
    if ((rc = debye_plan_create(&be, f_e.data(), c_e.data(), n_e.data(), 0, &plan.p))) return rc;
    debye_swarm sw{x.as<double>(), v.as<double>(), pbx.as<double>(), pbc.as<double>(), gbx.as<double>(),
                   gbc.as<double>(), gbi.as<int64_t>(), nullptr, 0, cost.as<double>(), nullptr};
    if ((rc = debye_pso_run(plan.p, &be, ld, d_lb.as<double>(), d_ub.as<double>(), p.pso, p.iters, damping, flags, &sw,
                            1, stream)))
      return rc;
    // polish each best, then its weights and error
    if (p.polish_steps > 0) {
      debye_lbfgs_params lp{p.polish_steps, 10, 30, 1e-4};
      debye_polish *pol = nullptr;
      if ((rc = debye_polish_create(&b1, f_e.data(), n_e.data(), ld, lp, &pol))) return rc;
      rc = debye_lbfgs_polish(pol, &b1, gbx.as<double>(), d_lb.as<double>(), d_ub.as<double>(), damping, flags,
                              nullptr, stream);
      debye_polish_destroy(pol);
      if (rc) return rc;
    }
    DevBuf w1, e1, c1, afe;
    if ((rc = alloc_doubles(w1, E * ld)) || (rc = alloc_doubles(e1, E)) || (rc = alloc_doubles(c1, E)) ||
        (rc = alloc_doubles(afe, E)))
      return rc;
    PlanHolder plan1;
    if ((rc = debye_plan_create(&b1, f_e.data(), one.data(), n_e.data(), 0, &plan1.p))) return rc;
    if ((rc = debye_fit_eval(plan1.p, &b1, gbx.as<double>(), ld, damping, flags, c1.as<double>(), w1.as<double>(),
                             e1.as<double>(), nullptr, stream)))
      return rc;
    if ((rc = debye_afe(&b1, gbx.as<double>(), ld, w1.as<double>(), e1.as<double>(), afe.as<double>(), stream)))
      return rc;
    std::vector<double> afe_h(E), einf_h(E);
    AUTO_HIP(hipMemcpyAsync(afe_h.data(), afe.p, (size_t)E * 8, hipMemcpyDeviceToHost, stream), "download");
    AUTO_HIP(hipMemcpyAsync(einf_h.data(), e1.p, (size_t)E * 8, hipMemcpyDeviceToHost, stream), "download");
    AUTO_HIP(hipStreamSynchronize(stream), "sync");

    // resolve: the smallest pole count of the round under the target; the
    // maximum pole count otherwise
    std::vector<int64_t> src_row, dst_row;
    std::vector<int32_t> rows_n;
    std::vector<int32_t> still;
    for (const int32_t m : unresolved) {
      const int64_t e0 = (int64_t)m * NN + (n0 - p.n_min);
      int64_t chosen = -1;
      for (int32_t k = 0; k < K; ++k)
        if (afe_h[e0 + k] < p.afe_target) {
          chosen = e0 + k;
          break;
        }
      if (chosen < 0 && n1 == p.n_max) chosen = e0 + (K - 1);
      if (chosen < 0) {
        still.push_back(m);
        continue;
      }
      src_row.push_back(chosen);
      dst_row.push_back(m);
      rows_n.push_back(n_e[chosen]);
      final_n[m] = n_e[chosen];
      final_einf[m] = einf_h[chosen];
      final_afe[m] = afe_h[chosen];
    }
    if (!src_row.empty()) {
      DevBuf d_sr, d_dr, d_rn;
      if ((rc = upload(d_sr, src_row, stream)) || (rc = upload(d_dr, dst_row, stream)) ||
          (rc = upload(d_rn, rows_n, stream)))
        return rc;
      const int64_t R = (int64_t)src_row.size();
      AUTO_HIP(dfit::launch_scatter_rows(R, d_sr.as<int64_t>(), d_dr.as<int64_t>(), d_rn.as<int32_t>(),
                                         gbx.as<double>(), ld, log10_tau_out, ld_out, stream),
               "scatter");
      AUTO_HIP(dfit::launch_scatter_rows(R, d_sr.as<int64_t>(), d_dr.as<int64_t>(), d_rn.as<int32_t>(),
                                         w1.as<double>(), ld, weights_out, ld_out, stream),
               "scatter");
      AUTO_HIP(hipStreamSynchronize(stream), "sync");
    }
    unresolved.swap(still);
  }
  AUTO_HIP(hipMemcpyAsync(n_poles_out, final_n.data(), (size_t)M * 4, hipMemcpyHostToDevice, stream), "upload");
  AUTO_HIP(hipMemcpyAsync(eps_inf_out, final_einf.data(), (size_t)M * 8, hipMemcpyHostToDevice, stream), "upload");
  AUTO_HIP(hipMemcpyAsync(afe_out, final_afe.data(), (size_t)M * 8, hipMemcpyHostToDevice, stream), "upload");
  AUTO_HIP(hipStreamSynchronize(stream), "sync");
  return DEBYE_OK;
}
