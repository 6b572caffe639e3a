// Internal interface between the C ABI layer and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

struct debye_plan;
struct debye_batch;

namespace dfit {

// Arguments of the cost / adjoint kernel (one work tile per 64-lane block).
struct FitArgs {
  const int64_t *f_off;
  const double *omega, *eps_re, *eps_im;
  const double *theta;
  int64_t ld;
  double damping;
  uint32_t flags;
  int32_t freq_split;     // SF: lanes per candidate along the frequency axis
  int32_t cand_per_wave;  // 64 / (SP * SF)
  int64_t n_tiles;        // work tiles (one per wavefront)
  // tiles of XCD x are xcd_off[x] .. xcd_off[x+1]-1 (in the order to run them)
  int64_t xcd_off[9];
  const int32_t *lane_cand;  // [tiles * cand_per_wave] candidate index or -1
  const int32_t *lane_mat;   // [tiles * cand_per_wave] material of that candidate
  double *cost, *weights, *eps_inf;
  int8_t *status;
  // adjoint
  const double *grad_cost;
  double *grad_theta;
  double *record;  // [n_cand][rec_ld] per-candidate w | z | mu | eps_inf, gc (or NULL)
  int64_t rec_ld;
  // [M] or NULL: materials whose candidates need no evaluation (nonzero);
  // a wave holding only such candidates exits at once, writing nothing
  const int32_t *skip_mat;
};

// One persistent launch over every pole-count bucket of a plan
// (fit_ragged.hip): per-bucket schedule fields, and the per-XCD lists of work
// items, each (bucket << 40) | tile, longest first.
struct RaggedBucket {
  int32_t n_poles, freq_split, cand_per_wave, uni;
  const int32_t *lane_cand, *lane_mat;
};
struct RaggedArgs {
  FitArgs common;                // batch, candidates, outputs (schedule fields per bucket)
  const RaggedBucket *buckets;   // [n_buckets]
  const int64_t *items;          // work items of XCD x: item_off[x] .. item_off[x+1]-1
  int64_t item_off[9];
  int32_t *counters;             // [8] next item of each XCD (reset by the launch)
};
hipError_t launch_fit_ragged(const RaggedArgs &r, int32_t blocks, size_t lds_bytes, hipStream_t s);

struct TargetGradArgs {
  const int64_t *f_off, *cand_off;
  const double *omega, *eps_re, *eps_im, *theta;
  int64_t ld;
  const double *record;
  int64_t rec_ld;
  const int32_t *mat_list;  // materials with this pole count
  double *grad_re, *grad_im;
};

int pole_split(int n_poles);
int lds_bytes_per_candidate(int n_poles);
// uni: every tile's active lanes belong to one material and the split is 1
hipError_t launch_fit(int n_poles, const FitArgs &a, int64_t n_tiles, bool grad, bool uni, hipStream_t s);
hipError_t launch_fit_grad(int n_poles, const FitArgs &a, int64_t n_tiles, bool uni, hipStream_t s);
hipError_t launch_fit_dd(int n_poles, const FitArgs &a, int64_t n_tiles, hipStream_t s);
hipError_t launch_target_grad(int n_poles, const TargetGradArgs &a, int64_t max_f, int32_t n_mats,
                              hipStream_t s);

// other kernels
struct MaterialArgs {
  int32_t M;
  const int8_t *kind;
  const double *params;
  const int64_t *f_off;
  int64_t n_freq;
  const double *omega;
  uint64_t noise_seed;
  double *eps_re, *eps_im, *jac;
};
hipError_t launch_material(const MaterialArgs &a, hipStream_t s);
hipError_t launch_material_vjp(int32_t M, const int64_t *f_off, const double *jac, const double *g_re,
                               const double *g_im, double *gp, hipStream_t s);

hipError_t launch_basis(const double *omega, int64_t F, const double *theta, int64_t ld, int64_t n_cand, int32_t N,
                        double *re, double *im, hipStream_t s);

struct PsoArgs {
  int32_t M;
  const int64_t *cand_off;
  const int32_t *n_poles;
  int64_t ld;
  const double *lb, *ub;
  double inertia, c1, c2;
  uint64_t seed;
  int32_t t, move;
  const int32_t *t_dev;  // if set, the iteration number is read from device memory
  const double *cost;
  double *x, *v, *pbest_x, *pbest_cost, *gbest_x, *gbest_cost;
  int64_t *gbest_idx;
  double *history;
  int64_t hist_ld;
};
hipError_t launch_pso_init(const PsoArgs &a, int64_t n_cand, hipStream_t s);
hipError_t launch_pso_step(const PsoArgs &a, hipStream_t s);
hipError_t launch_set_counter(int32_t *c, int32_t value, hipStream_t s);
// p[0..n) = v (a kernel, so that it can sit in a captured graph)
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_tick(int32_t *c, hipStream_t s);

// error text for debye_last_error() (api.hip); returns code
int set_error(int code, const char *msg);

// debye_fit_eval_grad with the target-gradient records in a buffer that the
// caller provides through record_buffer (api.hip; see there)
int fit_eval_grad_external(const debye_plan *p, const debye_batch *b, const double *log10_tau, int64_t ld,
                           double damping, uint32_t flags, const double *grad_cost, double *cost,
                           double *grad_log10_tau, double *grad_eps_re, double *grad_eps_im, int8_t *status,
                           int (*record_buffer)(size_t bytes, double **out), hipStream_t stream);

// average fractional error of fitted expansions (material.hip)
struct AfeArgs {
  int32_t M;
  const int64_t *f_off, *cand_off;
  const int32_t *n_poles;
  const double *omega, *eps_re, *eps_im;
  const double *theta, *weights, *eps_inf;
  int64_t ld;
  double *afe;
};
hipError_t launch_afe(const AfeArgs &a, int64_t n_cand, hipStream_t s);
hipError_t launch_gather_spectra(int64_t n_entries, const int64_t *src_off, const int32_t *src_mat,
                                 const int64_t *dst_off, const double *s0, const double *s1, const double *s2,
                                 double *d0, double *d1, double *d2, hipStream_t s);
hipError_t launch_scatter_rows(int64_t n_entries, const int64_t *src_row, const int64_t *dst_row, const int32_t *n,
                               const double *src, int64_t src_ld, double *dst, int64_t dst_ld, hipStream_t s);

// differential evolution (de.hip)
struct DeArgs {
  int32_t M;
  const int64_t *cand_off;
  const int32_t *n_poles;
  int64_t ld;
  const double *lb, *ub;
  double f_lo, f_hi, cr;
  uint64_t seed;
  int32_t t;
  const int32_t *t_dev;  // if set, the generation number is read from device memory
  double *x, *u;         // population and trial vectors [n_cand][ld]
  const double *cost_u;  // cost of the trials
  double *fit;           // cost of the members
  double *best_x, *best_cost;
  int64_t *best_idx;
  double *history;
  int64_t hist_ld;
};
hipError_t launch_de_init(const DeArgs &a, int64_t n_cand, hipStream_t s);
hipError_t launch_de_trial(const DeArgs &a, int64_t n_cand, hipStream_t s);
hipError_t launch_de_select(const DeArgs &a, hipStream_t s);

// annealing (da.hip)
struct DaArgs {
  int32_t M;
  const int64_t *cand_off;
  const int32_t *n_poles;
  int64_t ld;
  const double *lb, *ub;
  double qv, qa, t0;
  uint64_t seed;
  int32_t t;
  const int32_t *t_dev;  // if set, the generation number is read from device memory
  double *x, *u;         // chain states and proposals [n_cand][ld]
  const double *cost_u;  // cost of the proposals
  double *fit;           // cost of the states
  double *best_x, *best_cost;
  int64_t *best_idx;
  double *history;
  int64_t hist_ld;
};
hipError_t launch_da_init(const DaArgs &a, int64_t n_cand, hipStream_t s);
hipError_t launch_da_visit(const DaArgs &a, int64_t n_cand, hipStream_t s);
hipError_t launch_da_accept(const DaArgs &a, hipStream_t s);

struct LbfgsArgs {
  int32_t M;
  const int32_t *n_poles;
  int64_t ld;
  int32_t mem, max_trials;
  double c1;
  const double *lb, *ub;  // [M] search box
  double *theta;       // [M][ld] current point
  double *cost;        // [M] cost at theta
  double *grad;        // [M][ld] gradient at theta
  double *S, *Y;       // [M][mem][ld] history (ring)
  double *rho;         // [M][mem]
  int32_t *hist_n, *hist_head;  // [M]
  double *dir;         // [M][ld]
  double *gd;          // [M] g.d of the chosen direction
  // the trials of a step in three stages, rows of the trial arrays: the full
  // step of material m at row m; trials 1 .. ta at M + m*ta + (t-1); trials
  // ta+1 .. max_trials-1 at M + M*ta + m*tb + (t-1-ta), tb = max_trials-1-ta
  int32_t ta, tb;
  double *trial_theta; // [M*max_trials][ld]
  const double *trial_cost;  // [M*max_trials]
  const int8_t *trial_status;
  int32_t *done;       // [M] step decided (accepted a trial, or stalled)
  int32_t *stalled;    // [M] no acceptable trial at some step: the point never moves again
  double *new_theta;   // [M][ld] accepted point
  double *acc_cost;    // [M] cost of the accepted trial
  int32_t *accepted;   // [M]
  const double *new_cost, *new_grad;  // cost / gradient at new_theta
  const int8_t *new_status;
  double *cost_hist;   // [M][steps+1] or NULL
  int32_t step, steps;
};
hipError_t launch_lbfgs_direction(const LbfgsArgs &a, hipStream_t s);
hipError_t launch_lbfgs_first(const LbfgsArgs &a, hipStream_t s);
hipError_t launch_lbfgs_select(const LbfgsArgs &a, int32_t t_lo, int32_t t_hi, hipStream_t s);
hipError_t launch_lbfgs_update(const LbfgsArgs &a, hipStream_t s);

}  // namespace dfit
