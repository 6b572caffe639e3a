// Gradient polish of each material's best candidate: L-BFGS (Liu & Nocedal
// 1989) with the two-loop recursion (Nocedal & Wright, Algorithm 7.4) and
// Armijo backtracking alpha = 1, 1/2, 1/4, ... inside the search box: each
// trial point is projected onto [lb, ub] and the sufficient-decrease test uses
// the projected displacement p, C(trial) <= C + c1 min(g.p, 0) (clamping can
// make g.p positive; the cost is then not allowed to rise).  The accepted step
// is the first trial (largest alpha) that passes, which is what a sequential
// halving search returns.  The trials are evaluated in three batched cost
// launches: the full step of every material; then the next few halvings, only
// for the materials whose full step failed; then the rest, only for those
// still undecided (the waves of decided materials exit at once).  A step that
// accepts no trial leaves the point, gradient and history as they were, so
// every later step would rebuild and reject the same trials: such a material
// is marked stalled and left out of all later evaluations.  One thread per
// material.

#include "common.hpp"
#include "fit_eval.hpp"

namespace dfit {

// row of trial t of material m in the trial arrays (stage by stage)
__device__ __forceinline__ int64_t trial_row(const LbfgsArgs &a, int m, int t) {
  if (t == 0) return m;
  if (t <= a.ta) return (int64_t)a.M + (int64_t)m * a.ta + (t - 1);
  return (int64_t)a.M * (1 + a.ta) + (int64_t)m * a.tb + (t - 1 - a.ta);
}

__global__ __launch_bounds__(256) void lbfgs_direction_kernel(const LbfgsArgs a) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= a.M) return;
  const int N = a.n_poles[m];
  const int64_t ld = a.ld;
  const double *g = a.grad + (int64_t)m * ld;
  double *d = a.dir + (int64_t)m * ld;
  const double C = a.cost[m];
  if (a.cost_hist) a.cost_hist[(int64_t)m * (a.steps + 1) + a.step] = C;
  bool skip = !(fabs(C) < INFINITY);
  for (int i = 0; i < N; ++i) skip = skip || !(fabs(g[i]) < INFINITY);
  double gd = 0.0;
  if (!skip) {
    const int mem = a.mem;
    int n = a.hist_n[m];
    const int head = a.hist_head[m];
    double q[DFIT_MAX_POLES], alpha[DFIT_MAX_MEM];
    for (int i = 0; i < N; ++i) q[i] = g[i];
    // newest to oldest
    for (int j = n - 1; j >= 0; --j) {
      const int slot = (head - n + j + mem) % mem;
      const double *s = a.S + ((int64_t)m * mem + slot) * ld;
      const double *y = a.Y + ((int64_t)m * mem + slot) * ld;
      double t = 0.0;
      for (int i = 0; i < N; ++i) t += s[i] * q[i];
      alpha[j] = a.rho[(int64_t)m * mem + slot] * t;
      for (int i = 0; i < N; ++i) q[i] -= alpha[j] * y[i];
    }
    double gamma = 1.0;
    if (n > 0) {
      const int slot = (head - 1 + mem) % mem;
      const double *s = a.S + ((int64_t)m * mem + slot) * ld;
      const double *y = a.Y + ((int64_t)m * mem + slot) * ld;
      double sy = 0.0, yy = 0.0;
      for (int i = 0; i < N; ++i) {
        sy += s[i] * y[i];
        yy += y[i] * y[i];
      }
      gamma = sy / yy;
    }
    for (int i = 0; i < N; ++i) q[i] *= gamma;
    for (int j = 0; j < n; ++j) {
      const int slot = (head - n + j + mem) % mem;
      const double *s = a.S + ((int64_t)m * mem + slot) * ld;
      const double *y = a.Y + ((int64_t)m * mem + slot) * ld;
      double t = 0.0;
      for (int i = 0; i < N; ++i) t += y[i] * q[i];
      const double b = a.rho[(int64_t)m * mem + slot] * t;
      for (int i = 0; i < N; ++i) q[i] += (alpha[j] - b) * s[i];
    }
    for (int i = 0; i < N; ++i) {
      d[i] = -q[i];
      gd += g[i] * d[i];
    }
    if (n == 0 || !(gd < 0.0)) {
      // steepest descent, largest component at most one decade
      a.hist_n[m] = 0;
      double gmax = 0.0;
      for (int i = 0; i < N; ++i) gmax = fmax(gmax, fabs(g[i]));
      if (!(gmax > 0.0)) {
        skip = true;
      } else {
        const double sc = fmin(1.0, 1.0 / gmax);
        gd = 0.0;
        for (int i = 0; i < N; ++i) {
          d[i] = -g[i] * sc;
          gd += g[i] * d[i];
        }
      }
    }
  }
  a.gd[m] = skip ? NAN : gd;
  const double *th = a.theta + (int64_t)m * ld;
  const double lo = a.lb[m], hi = a.ub[m];
  double alpha_t = 1.0;
  for (int t = 0; t < a.max_trials; ++t) {
    double *tt = a.trial_theta + trial_row(a, m, t) * ld;
    for (int i = 0; i < N; ++i) {
      const double v = th[i] + alpha_t * d[i];
      tt[i] = skip ? th[i] : (v < lo ? lo : (v > hi ? hi : v));
    }
    alpha_t *= 0.5;
  }
}

namespace {
// the sufficient-decrease test of trial t of material m
__device__ bool armijo_ok(const LbfgsArgs &a, int m, int t, double cost_t, int8_t status_t) {
  const int N = a.n_poles[m];
  const double *g = a.grad + (int64_t)m * a.ld;
  const double *th = a.theta + (int64_t)m * a.ld;
  const double *tt = a.trial_theta + trial_row(a, m, t) * a.ld;
  double gp = 0.0;
  for (int i = 0; i < N; ++i) gp += g[i] * (tt[i] - th[i]);
  return status_t == ST_OK && cost_t <= a.cost[m] + a.c1 * fmin(gp, 0.0);
}

// the step's outcome: trial `pick` accepted with cost `c`, or none (pick < 0)
__device__ void decide(const LbfgsArgs &a, int m, int pick, double c) {
  const int N = a.n_poles[m];
  a.accepted[m] = pick >= 0 ? 1 : 0;
  a.acc_cost[m] = pick >= 0 ? c : a.cost[m];
  const double *src = pick >= 0 ? a.trial_theta + trial_row(a, m, pick) * a.ld : a.theta + (int64_t)m * a.ld;
  for (int i = 0; i < N; ++i) a.new_theta[(int64_t)m * a.ld + i] = src[i];
}
}  // namespace

// after the first launch: materials whose full step passes (or that are
// skipped) are decided; the rest wait for the remaining trials
__global__ __launch_bounds__(256) void lbfgs_first_kernel(const LbfgsArgs a) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= a.M) return;
  const double gd = a.gd[m];
  // stalled earlier (its full step was not evaluated), or nothing to step
  // along (non-finite cost or gradient, zero gradient): no step
  if (a.stalled[m] || !(gd == gd)) {
    decide(a, m, -1, 0.0);
    a.done[m] = 1;
    a.stalled[m] = 1;
    return;
  }
  if (armijo_ok(a, m, 0, a.trial_cost[m], a.trial_status[m])) {
    decide(a, m, 0, a.trial_cost[m]);
    a.done[m] = 1;
    return;
  }
  a.done[m] = 0;
  if (a.max_trials == 1) {
    decide(a, m, -1, 0.0);
    a.stalled[m] = 1;
  }
}

// after the launch of trials t_lo .. t_hi: the first of them that passes, for
// the materials still undecided; after the last stage, no pass is a stall
__global__ __launch_bounds__(256) void lbfgs_select_kernel(const LbfgsArgs a, int32_t t_lo, int32_t t_hi) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= a.M || a.done[m]) return;
  for (int t = t_lo; t <= t_hi; ++t) {
    const int64_t r = trial_row(a, m, t);
    if (armijo_ok(a, m, t, a.trial_cost[r], a.trial_status[r])) {
      decide(a, m, t, a.trial_cost[r]);
      a.done[m] = 1;
      return;
    }
  }
  if (t_hi == a.max_trials - 1) {
    decide(a, m, -1, 0.0);
    a.done[m] = 1;
    a.stalled[m] = 1;
  }
}

__global__ __launch_bounds__(256) void lbfgs_update_kernel(const LbfgsArgs a) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= a.M) return;
  const int N = a.n_poles[m];
  const int64_t ld = a.ld;
  if (a.accepted[m]) {
    const int mem = a.mem;
    const int head = a.hist_head[m];
    // the pair is formed in registers and stored only if it is kept: with a
    // full history, slot `head` still holds the oldest live pair, which a
    // rejected pair (s.y <= 1e-300) must not overwrite
    double s[DFIT_MAX_POLES], y[DFIT_MAX_POLES];
    double sy = 0.0;
    for (int i = 0; i < N; ++i) {
      s[i] = a.new_theta[m * ld + i] - a.theta[m * ld + i];
      y[i] = a.new_grad[m * ld + i] - a.grad[m * ld + i];
      sy += s[i] * y[i];
    }
    if (sy > 1e-300) {
      double *ss = a.S + ((int64_t)m * mem + head) * ld;
      double *yy = a.Y + ((int64_t)m * mem + head) * ld;
      for (int i = 0; i < N; ++i) {
        ss[i] = s[i];
        yy[i] = y[i];
      }
      a.rho[(int64_t)m * mem + head] = 1.0 / sy;
      a.hist_head[m] = (head + 1) % mem;
      a.hist_n[m] = a.hist_n[m] < mem ? a.hist_n[m] + 1 : mem;
    }
    for (int i = 0; i < N; ++i) {
      a.theta[m * ld + i] = a.new_theta[m * ld + i];
      a.grad[m * ld + i] = a.new_grad[m * ld + i];
    }
    a.cost[m] = a.acc_cost[m];  // the evaluation the acceptance test used
  }
  if (a.cost_hist && a.step == a.steps - 1) a.cost_hist[(int64_t)m * (a.steps + 1) + a.steps] = a.cost[m];
}

static dim3 grid_for(int32_t M) { return dim3((unsigned)((M + 255) / 256)); }

hipError_t launch_lbfgs_direction(const LbfgsArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(lbfgs_direction_kernel, grid_for(a.M), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_lbfgs_first(const LbfgsArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(lbfgs_first_kernel, grid_for(a.M), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_lbfgs_select(const LbfgsArgs &a, int32_t t_lo, int32_t t_hi, hipStream_t s) {
  hipLaunchKernelGGL(lbfgs_select_kernel, grid_for(a.M), dim3(256), 0, s, a, t_lo, t_hi);
  return hipGetLastError();
}
hipError_t launch_lbfgs_update(const LbfgsArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(lbfgs_update_kernel, grid_for(a.M), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace dfit
