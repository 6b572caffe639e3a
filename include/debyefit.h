/*
 * debyefit.h - C ABI of the MI355X (gfx950) library for the batched
 * multi-pole Debye fitting method of Majchrowska, Giannakis, Warren and
 * Giannopoulos, "Modelling Arbitrary Complex Dielectric Properties - an
 * automated implementation for gprMax" (2021).
 *
 * The method (Sec. III-B) fits  eps(w) = eps_inf + sum_n d_eps_n / (1 + j w tau_n)
 * (Eq. 7, with eps = eps' - j eps'' as in Eq. 1) to a target spectrum.  A
 * global optimiser searches the relaxation times; for every candidate set
 * the pole weights come from a damped least-squares (DLS) fit to the loss
 * part eps'', negative weights are flipped to positive as a penalty, eps_inf
 * is the mean real-part misfit and the cost is the sum of squared real and
 * imaginary residuals over the frequency points.
 *
 * Conventions for every entry point
 *  - All array pointers are DEVICE pointers unless the name ends in _host.
 *    The caller owns every buffer; the library neither frees nor keeps them
 *    after the call returns (a plan keeps only its own buffers).
 *  - Calls enqueue work on `stream` and return without synchronising.
 *  - Return value: DEBYE_OK (0) or a negative DEBYE_E* code.  Argument errors
 *    are detected on the host before anything is enqueued; the message is
 *    available from debye_last_error() (per thread).
 *  - Numerical trouble is reported per candidate in `status` (DEBYE_ST_*).
 *  - FP64 throughout.
 *  - Candidate log10(tau) values and weights are stored in rows of stride
 *    `ld` (>= the material's pole count); only the first n_poles[m] entries of
 *    a row are read or written.
 */
#ifndef DEBYEFIT_H
#define DEBYEFIT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DEBYE_MAX_POLES 24

/* return codes */
enum {
  DEBYE_OK = 0,
  DEBYE_EINVAL = -1, /* NULL pointer, unknown enum value, shape mismatch */
  DEBYE_ERANGE = -2, /* size out of range: M < 1, F < 1, N < 1 or N > DEBYE_MAX_POLES,
                        ld < N, damping < 0 or not finite */
  DEBYE_EHIP = -3,   /* HIP runtime / launch failure (text in debye_last_error) */
  DEBYE_ENOMEM = -4  /* device allocation inside a plan failed */
};

/* per-candidate status */
enum {
  DEBYE_ST_OK = 0,
  DEBYE_ST_BADINPUT = 1, /* non-finite log10(tau), |log10 tau| > 30, or non-finite
                            omega / eps' / eps'' of the material: cost = NaN */
  DEBYE_ST_SINGULAR = 2  /* the scaled damped normal matrix is numerically singular
                            (only reachable with damping ~ 0, e.g. duplicate
                            relaxation times): cost = +Inf, weights = NaN */
};

/* flags */
enum {
  DEBYE_FLAG_NO_SIGN_FLIP = 1u, /* keep signed LS weights (w = z instead of |z|) */
  DEBYE_FLAG_NO_REFINE = 2u,    /* skip the refinement step (one corrected
                                   semi-normal-equations pass, Sec. III-B's damped
                                   least squares solved to full accuracy): z is the
                                   damped Cholesky solution of the normal equations
                                   alone.  Faster (one basis pass fewer in the
                                   forward evaluation), but its relative error in z
                                   grows with the condition number of the scaled
                                   damped Gram matrix (at most about
                                   n_poles / damping) times the unit roundoff, so
                                   costs are no longer within 1e-10 of the
                                   least-squares result for ill-conditioned
                                   candidates.  In debye_fit_eval_grad the
                                   gradient formula then holds only to that error. */
  DEBYE_FLAG_DD_REFINE = 4u     /* the refinement step in double-double arithmetic
                                   (relaxation times 10^theta, the basis, the
                                   residual eps'' - I z and the sums I^T r to about
                                   104 bits): the cost is then within about 1e-11 of
                                   the exact least-squares result also on the rare
                                   ill-conditioned candidates (a few in 10^6 of
                                   random ones) where the FP64 refinement's basis
                                   and residual roundings leave up to a few 1e-10.
                                   Slower (the refinement pass costs about five
                                   times the FP64 one: 2 to 3 times the forward
                                   kernel's time).  Forward evaluations only
                                   (debye_fit_eval and the optimisers' runs, which
                                   then use one launch per pole-count bucket);
                                   DEBYE_EINVAL together with DEBYE_FLAG_NO_REFINE,
                                   in debye_fit_eval_grad, in the polish calls and
                                   in debye_fit_auto with polish steps. */
};

/* material kinds for debye_material_eval (parameter rows of DEBYE_PARAM_STRIDE) */
enum {
  DEBYE_KIND_DEBYE = 0,    /* Eq. 3: (eps_inf, d_eps, tau0) */
  DEBYE_KIND_HN = 1,       /* Eq. 4: (eps_inf, d_eps, tau0, alpha, beta) */
  DEBYE_KIND_CC = 2,       /* Eq. 4 with beta = 1 (Cole-Cole): params[4] ignored */
  DEBYE_KIND_CD = 3,       /* Eq. 4 with alpha = 1 (Cole-Davidson): params[3] ignored */
  DEBYE_KIND_JONSCHER = 4, /* (eps_inf, chi, omega_p, n): eps_inf + chi (j w / omega_p)^(n-1) */
  DEBYE_KIND_CRIM = 5,     /* Eq. 6 with a = 1/2: Debye water phase (eps_inf_w, d_eps_w,
                              tau_w) at volume fraction f_w in a lossless matrix eps_m:
                              (eps_inf_w, d_eps_w, tau_w, f_w, eps_m) */
  DEBYE_KIND_HNSUM = 6     /* tabulated-style data: eps_inf + up to three HN terms,
                              (eps_inf, n_terms, [d_eps, tau0, alpha, beta] x 3 at
                              params[2..13], noise at params[14]); values are multiplied
                              by (1 + noise * g) with g standard normal (Box-Muller on
                              Philox4x64-10, key (noise_seed, m), counter (k, 0, 0, 2)) */
};
#define DEBYE_PARAM_STRIDE 16

/* ------------------------------------------------------------------------
 * Ragged batch of materials.  Material m owns frequency points
 * [f_off[m], f_off[m+1]) of omega/eps_re/eps_im and candidates
 * [cand_off[m], cand_off[m+1]); it is fitted with n_poles[m] poles.
 * ------------------------------------------------------------------------ */
typedef struct debye_batch {
  int32_t n_mat;           /* M >= 1 */
  int32_t max_poles;       /* max_m n_poles[m] (host value), 1..DEBYE_MAX_POLES */
  int64_t n_freq;          /* f_off[M] (host value) */
  int64_t n_cand;          /* cand_off[M] (host value) */
  const int64_t *f_off;    /* [M+1] device */
  const int64_t *cand_off; /* [M+1] device */
  const int32_t *n_poles;  /* [M]   device */
  const double *omega;     /* [n_freq] angular frequency 2 pi f (rad/s), 0 < omega < 1e45 */
  const double *eps_re;    /* [n_freq] eps'  */
  const double *eps_im;    /* [n_freq] eps'' (loss, >= 0 for passive media) */
} debye_batch;

/* A plan holds the launch schedule for one batch shape: candidates grouped by
 * pole count, lanes per candidate, work lists sorted by cost (longest first),
 * and workspace.  Build it once per shape from HOST copies of the offsets;
 * reuse it for every call on batches of that shape (e.g. every iteration of
 * an optimiser).  `flags`: 0, or DEBYE_PLAN_TARGET_GRAD to also allocate the
 * per-candidate adjoint records that debye_fit_eval_grad needs for target
 * gradients (n_cand x (4 max_poles + 2) doubles).  Every buffer a plan uses
 * is allocated here, so the evaluation calls never allocate.
 * With more than one pole count the buckets of an evaluation are forked from
 * the caller's stream onto up to four streams owned by the plan and joined
 * back before the call's work is complete on the caller's stream (under
 * stream capture they become parallel graph branches).  A plan is therefore
 * not to be used from two host threads at once. */
typedef struct debye_plan debye_plan;

/* plan flags */
enum {
  DEBYE_PLAN_TARGET_GRAD = 1u /* workspace for the target gradients of debye_fit_eval_grad */
};

int debye_plan_create(const debye_batch *shape, const int64_t *f_off_host, const int64_t *cand_off_host,
                      const int32_t *n_poles_host, uint32_t flags, debye_plan **out);
int debye_plan_destroy(debye_plan *plan);

/* Override the schedule's frequency split (lanes per candidate along the
 * frequency axis, a power of two; 0 restores the automatic choice) for pole
 * count n_poles (0 = all). Used by the autotuner and the tests.  Re-tiling
 * (here or in debye_plan_autotune) makes the plan's next optimiser run
 * re-capture its graph.  Not while work of the plan is in flight. */
int debye_plan_set_freq_split(debye_plan *plan, int32_t n_poles, int32_t split);

/* How an evaluation of a plan with several pole counts is launched:
 *   DEBYE_LAUNCH_BUCKETS:    one launch per pole-count bucket, forked onto the
 *                            plan's streams and joined (the default);
 *   DEBYE_LAUNCH_PERSISTENT: one persistent launch over every bucket: a fixed
 *                            grid of one-wave blocks, eight per CU, each taking
 *                            work items (a bucket's tile) from its XCD's list,
 *                            longest estimated duration first, through a
 *                            counter in device memory, until the list is empty;
 *   DEBYE_LAUNCH_AUTO:       back to the default, and let debye_plan_autotune
 *                            time both and keep the faster.
 * Plans with one pole count always launch it directly.  The forward
 * evaluation (debye_fit_eval and the optimisers' runs) uses the mode; the
 * adjoint keeps the per-bucket launches.  Not while work of the plan is in
 * flight.  debye_plan_get_launch returns the mode in use (>= 0) or an error. */
enum { DEBYE_LAUNCH_AUTO = 0, DEBYE_LAUNCH_BUCKETS = 1, DEBYE_LAUNCH_PERSISTENT = 2 };
int debye_plan_set_launch(debye_plan *plan, int32_t mode);
int debye_plan_get_launch(const debye_plan *plan);

/* Autotune the schedule on real data: for every pole-count bucket without an
 * override, time `reps` launches (1..100) of the cost kernel at each frequency
 * split (1, 2, 4, ... up to 64 / pole split, while spectra keep at least 8
 * points per lane) with HIP events on `stream`, after about 30 ms of warm-up
 * launches and in three rounds (the best time of each split counts), and keep
 * the fastest (a wider split must be at least 3 % faster than the best
 * narrower one).  The
 * arguments are those of debye_fit_eval (log10_tau: a representative set of
 * candidates, e.g. the initial swarm).  Synchronises `stream`; allocates and
 * frees a temporary cost buffer, so it is a set-up call, not for capture.
 * The choice stays in the plan (debye_plan_info reports it); an override set
 * by debye_plan_set_freq_split takes precedence.  With several pole counts
 * (and no mode fixed by debye_plan_set_launch) it then times whole
 * evaluations with both launch modes, three rounds of `reps`, and keeps the
 * persistent launch if it is at least 3 % faster. */
int debye_plan_autotune(debye_plan *plan, const debye_batch *b, const double *log10_tau, int64_t ld,
                        double damping, uint32_t flags, int32_t reps, hipStream_t stream);

/* Host-only preview of the work tiles a plan builds for one pole-count
 * bucket (no device call; for inspection and tests).  f_off, cand_off: the
 * batch's HOST offsets; mats [n_mats]: the bucket's materials (all with
 * n_poles poles).  With lane_cand and lane_mat non-NULL (capacity entries
 * each) it writes every wave's slots, 64 / (pole_split * freq_split) per
 * tile, candidate index or -1 and its material; xcd_off [9]: the tiles of
 * XCD x are xcd_off[x] .. xcd_off[x+1]-1; *uniform: 1 when every tile's
 * candidates belong to one material (the kernels then read the spectra with
 * wave-uniform addresses).  Returns the number of slots (>= 0) or a negative
 * error code. */
int debye_schedule_preview(const int64_t *f_off, const int64_t *cand_off, const int32_t *mats, int32_t n_mats,
                           int32_t n_poles, int32_t pole_split, int32_t freq_split, int32_t *lane_cand,
                           int32_t *lane_mat, int64_t capacity, int64_t *xcd_off, int32_t *uniform);

/* Schedule introspection: with i < 0 returns the number of pole-count buckets;
 * otherwise fills the pole count, pole split, frequency split, number of work
 * tiles of bucket i and whether its tiles are uniform (one material per wave;
 * see debye_schedule_preview).  Any output pointer may be NULL. */
int debye_plan_info(const debye_plan *plan, int32_t i, int32_t *n_poles, int32_t *pole_split, int32_t *freq_split,
                    int64_t *n_tiles, int32_t *uniform);

/* Text of the last error on this thread ("" if none). */
const char *debye_last_error(void);

/* Library version string. */
const char *debye_version(void);

/* ------------------------------------------------------------------------
 * Debye basis (Eq. 7 split by Eq. 1): for every candidate c and pole i,
 *   x = omega[k] * 10^log10_tau[c*ld+i],  re[(c*N+i)*F+k] = 1/(1+x^2),
 *   im[(c*N+i)*F+k] = x/(1+x^2).
 * omega [F], log10_tau [n_cand][ld], re/im [n_cand][N][F].
 * ------------------------------------------------------------------------ */
int debye_basis(const double *omega, int64_t F, const double *log10_tau, int64_t ld, int64_t n_cand,
                int32_t N, double *re, double *im, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Cost evaluation (Sec. III-B), one result per candidate c of material m:
 *   tau_i = 10^log10_tau[c*ld+i]; R_ki = 1/(1+x^2), I_ki = x/(1+x^2), x = w_k tau_i
 *   z   = argmin || I z - eps'' ||^2 + damping * sum_i (||I_:,i|| z_i)^2
 *         (damped least squares with Marquardt column scaling)
 *   w_i = |z_i|  (unless DEBYE_FLAG_NO_SIGN_FLIP)
 *   eps_inf = mean_k (eps'_k - sum_i w_i R_ki)
 *   cost = sum_k (eps'_k - eps_inf - sum_i w_i R_ki)^2 + (eps''_k - sum_i w_i I_ki)^2
 * Outputs (each may be NULL except cost): cost [n_cand], weights [n_cand][ld]
 * (the fitted d_eps_i = w_i), eps_inf [n_cand], status [n_cand].
 * damping >= 0 (1e-8 is the library default used by the optimisers).
 * ------------------------------------------------------------------------ */
int debye_fit_eval(const debye_plan *plan, const debye_batch *b, const double *log10_tau, int64_t ld,
                   double damping, uint32_t flags, double *cost, double *weights, double *eps_inf,
                   int8_t *status, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Cost and its variable-projection adjoint.  With M = I^T I + damping diag(I^T I),
 * M z = I^T eps'', s = sign(z) (1 without the flip), r', r'' the residuals:
 *   g_w = -2 (R^T r' + I^T r''),  mu = M^-1 (s o g_w)
 *   dC/dlog10tau_i = -2 w_i (dR_i.r' + dI_i.r'') + mu_i dI_i.(eps'' - I z)
 *                    - z_i dI_i.(I mu) - 2 damping mu_i z_i dI_i.I_i
 *   dC/deps'_k = 2 r'_k,  dC/deps''_k = 2 r''_k + (I mu)_k
 * (dR/dlog10tau = -2 ln10 x^2 R^2, dI/dlog10tau = ln10 x R^2 (1 - x^2)).
 * grad_cost [n_cand] (NULL = all ones) scales each candidate.
 * grad_log10_tau [n_cand][ld] receives grad_cost[c] * dC/dlog10tau.
 * grad_eps_re / grad_eps_im [n_freq] (both NULL or both set) receive the target
 * gradients summed over the candidates of each material (fixed order, so the
 * result is deterministic); they need a plan created with
 * DEBYE_PLAN_TARGET_GRAD (DEBYE_EINVAL otherwise).  Padding entries of a row
 * (i >= n_poles[m]) of grad_log10_tau are set to 0.
 * ------------------------------------------------------------------------ */
int debye_fit_eval_grad(const debye_plan *plan, const debye_batch *b, const double *log10_tau, int64_t ld,
                        double damping, uint32_t flags, const double *grad_cost, double *cost,
                        double *grad_log10_tau, double *grad_eps_re, double *grad_eps_im, int8_t *status,
                        hipStream_t stream);

/* ------------------------------------------------------------------------
 * debye_fit_eval_grad for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results, but the target
 * gradients need no DEBYE_PLAN_TARGET_GRAD plan.  Their per-candidate records
 * live in a static 64 MiB device array of the library (one per GPU, held
 * until the process ends), so n_cand x (4 max_poles + 2) x 8 bytes must not
 * exceed 64 MiB (DEBYE_ERANGE otherwise, checked on the host before any
 * work is enqueued).  Every call on a GPU shares that array: calls that
 * overlap on one GPU (other streams or threads) race.  The call itself
 * allocates nothing; the plan is made beforehand.
 * ------------------------------------------------------------------------ */
int debye_fit_eval_grad_noalloc(const debye_plan *plan, const debye_batch *b, const double *log10_tau, int64_t ld,
                                double damping, uint32_t flags, const double *grad_cost, double *cost,
                                double *grad_log10_tau, double *grad_eps_re, double *grad_eps_im, int8_t *status,
                                hipStream_t stream);

/* ------------------------------------------------------------------------
 * Target synthesis (Eqs. 3-6): eps_re/eps_im [n_freq] for every material
 * (kind [M] int8, params [M][DEBYE_PARAM_STRIDE]); jac (NULL or [n_freq][5][2])
 * receives d(eps', eps'')/d(eps_inf, d_eps, tau0, alpha, beta) for the
 * Debye/HN/CC/CD kinds (NaN for the others).
 * ------------------------------------------------------------------------ */
int debye_material_eval(int32_t M, const int8_t *kind, const double *params, const int64_t *f_off,
                        int64_t n_freq, const double *omega, uint64_t noise_seed, double *eps_re,
                        double *eps_im, double *jac, hipStream_t stream);

/* Material-parameter gradient (chain rule through Eq. 4): for every material
 * m, grad_params[m][q] = sum_k jac[k][q][0] grad_re[k] + jac[k][q][1] grad_im[k]
 * over its frequency points, q = eps_inf, d_eps, tau0, alpha, beta; entries
 * 5..15 of each row are set to 0.  jac as produced by debye_material_eval;
 * grad_re/grad_im [n_freq] (e.g. the target gradients of debye_fit_eval_grad);
 * grad_params [M][DEBYE_PARAM_STRIDE].  Deterministic (fixed reduction order). */
int debye_material_vjp(int32_t M, const int64_t *f_off, int64_t n_freq, const double *jac, const double *grad_re,
                       const double *grad_im, double *grad_params, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Particle swarm over log10(tau), one swarm per material (Sec. III-A/B: PSO
 * for the relaxation times, Kennedy & Eberhart).  Random numbers are
 * Philox4x64-10 (Salmon et al. 2011) words with key (seed, m) and counter
 * (dimension, particle, iteration, stream), u = (word >> 11) * 2^-53.
 *
 * pso_init: x = lb + (ub-lb) u0, v = (ub-lb)(2 u1 - 1) from counter (d, p, 0, 0);
 *   pbest_x = x; pbest_cost = +Inf; gbest_cost = +Inf; gbest_idx = -1.
 * pso_step (after `cost` = f(x) for the whole swarm), iteration t >= 1:
 *   pbest updated where cost < pbest_cost (strictly; NaN never wins);
 *   the lowest-index minimum of pbest_cost replaces the global best if strictly
 *   better; history[m*hist_ld + t-1] = gbest_cost[m] (history may be NULL);
 *   if move: r1, r2 from counter (d, p, t, 1),
 *     v = ((inertia*v) + ((c1*r1)*(pbest-x))) + ((c2*r2)*(gbest-x))
 *     (the social term is omitted while gbest_idx < 0), x = clamp(x + v, lb, ub).
 *   Evaluation order is fixed and no fused multiply-add is used, so results
 *   are bit-reproducible.
 * lb, ub [M]; x, v, pbest_x [n_cand][ld]; pbest_cost [n_cand];
 * gbest_x [M][ld]; gbest_cost [M]; gbest_idx [M] (index within the material).
 * ------------------------------------------------------------------------ */
typedef struct debye_pso_params {
  double inertia, c1, c2;
  uint64_t seed;
} debye_pso_params;

int debye_pso_init(const debye_batch *b, int64_t ld, const double *lb, const double *ub, debye_pso_params p,
                   double *x, double *v, double *pbest_x, double *pbest_cost, double *gbest_cost,
                   int64_t *gbest_idx, hipStream_t stream);
int debye_pso_step(const debye_batch *b, int64_t ld, const double *lb, const double *ub, debye_pso_params p,
                   int32_t t, int32_t move, const double *cost, double *x, double *v, double *pbest_x,
                   double *pbest_cost, double *gbest_x, double *gbest_cost, int64_t *gbest_idx,
                   double *history, int64_t hist_ld, hipStream_t stream);

/* ------------------------------------------------------------------------
 * A whole swarm fit: pso_init, cost evaluation, then `iters` x (pso_step with
 * move, cost evaluation), then a bests-only pso_step; P*(iters+1) evaluations
 * per material.  With use_graph != 0 one iteration (step -> evaluation ->
 * iteration-counter increment) is captured once as a HIP graph (kept in the
 * plan and reused while the arguments are unchanged) and replayed `iters`
 * times on a stream owned by the plan, ordered after and before `stream` by
 * events; results are bit-identical to use_graph = 0.  history needs
 * hist_ld >= iters + 1.  Calls with one plan must not overlap.
 * ------------------------------------------------------------------------ */
typedef struct debye_swarm {
  double *x, *v, *pbest_x;          /* [n_cand][ld] */
  double *pbest_cost;               /* [n_cand] */
  double *gbest_x;                  /* [M][ld] */
  double *gbest_cost;               /* [M] */
  int64_t *gbest_idx;               /* [M] */
  double *history;                  /* [M][hist_ld] or NULL */
  int64_t hist_ld;
  double *cost;                     /* [n_cand] cost of the current positions (workspace/output) */
  int8_t *status;                   /* [n_cand] or NULL */
} debye_swarm;

int debye_pso_run(const debye_plan *plan, const debye_batch *b, int64_t ld, const double *lb, const double *ub,
                  debye_pso_params p, int32_t iters, double damping, uint32_t flags, const debye_swarm *swarm,
                  int32_t use_graph, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Average fractional error of fitted expansions (the paper's accuracy figure,
 * Sec. IV, Table I), in percent, per candidate:
 *   100 (mean_k |eps'_k - m'_k| / |eps'_k| + mean_k |eps''_k - m''_k| / |eps''_k|)
 * with the model m = eps_inf + sum_i w_i / (1 + j omega_k tau_i) (m'' its loss,
 * sign of Eq. 1) and points where eps'' = 0 left out of the second mean.
 * log10_tau, weights: [n_cand][ld]; eps_inf, afe: [n_cand] (device).
 * ------------------------------------------------------------------------ */
int debye_afe(const debye_batch *b, const double *log10_tau, int64_t ld, const double *weights,
              const double *eps_inf, double *afe, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Automatic number of poles (Sec. III-B: with the pole count set to -1 the
 * fit starts from one pole and adds poles until the average fractional error
 * drops below 5 % or 20 poles are reached).  Batched over materials: the
 * materials still unresolved are fitted with the next `chunk` pole counts at
 * once, as one ragged batch in which every (material, N) pair is an entry with
 * its own swarm of `particles` (Philox key (seed, entry index), entries
 * ordered material-major, N ascending); each swarm best is polished
 * (`polish_steps` L-BFGS steps, memory 10, 30 trials, c1 = 1e-4) and its AFE
 * computed.  A material is resolved at the smallest N of the round whose AFE
 * is below afe_target; materials that reach n_max keep the n_max fit.  The
 * result is the pole count that the one-at-a-time procedure would stop at for
 * these per-entry swarms; `chunk` only trades extra fits for fewer rounds.
 *   mats: spectra of the M materials (n_mat, n_freq, f_off, omega, eps_re,
 *         eps_im are used; the other fields are ignored); f_off_host its host
 *         copy; lb, ub: device [M] bounds of log10 tau.
 *   outputs (device): n_poles_out [M], log10_tau_out and weights_out
 *         [M][ld_out] (ld_out >= n_max; entries past n_poles_out[m] are left
 *         unchanged), eps_inf_out [M], afe_out [M].
 * Allocates its own workspace, synchronises `stream` after every round.
 * ------------------------------------------------------------------------ */
typedef struct debye_auto_params {
  int32_t n_min, n_max;     /* 1 <= n_min <= n_max <= DEBYE_MAX_POLES (the paper: 1 .. 20) */
  int32_t chunk;            /* pole counts fitted per round, >= 1 */
  double afe_target;        /* percent (the paper: 5) */
  int32_t particles, iters; /* swarm of each (material, N): >= 1 particles, >= 0 iterations */
  debye_pso_params pso;
  int32_t polish_steps;     /* >= 0 */
} debye_auto_params;

int debye_fit_auto(const debye_batch *mats, const int64_t *f_off_host, const double *lb, const double *ub,
                   debye_auto_params p, double damping, uint32_t flags, int32_t *n_poles_out,
                   double *log10_tau_out, double *weights_out, double *eps_inf_out, double *afe_out,
                   int64_t ld_out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Differential evolution (the paper's DE-DLS alternative, Sec. III-A; Storn &
 * Price 1997, strategy rand/1/bin), one population per material over log10
 * tau: the candidates of material m are its members.  Generation-synchronous:
 * every trial of generation t >= 1 is built from the population as it stood
 * before the generation, the trials are evaluated together, and member i is
 * replaced by its trial when cost(trial) <= cost(member) (a NaN cost never
 * replaces).  Trial i: donors r1, r2, r3 distinct and != i, drawn uniformly;
 * mutant x_r1 + F (x_r2 - x_r3) (each operation rounded separately) with
 * F = f_lo + (f_hi - f_lo) u drawn once per material and generation
 * (dither); binomial crossover with rate cr and one forced coordinate; a
 * crossed coordinate outside [lb[m], ub[m]] is redrawn uniformly in the box.
 * A population of fewer than 4 members is not evolved (trial = target).
 * Random numbers: Philox4x64-10, key (seed, material); the counters are
 * listed in the library source.  Fed the same costs, runs are bit-identical
 * to the CPU reference.
 *   debye_de_init:   x uniform in the box; fit = +inf; best_cost = +inf,
 *                    best_idx = -1.
 *   debye_de_trial:  u = trials of generation t from x.
 *   debye_de_select: greedy replacement with cost_u = cost(u); then the
 *                    material's best (lowest index among equal costs) if it
 *                    improves; history[m * hist_ld + t] = best cost (may be
 *                    NULL).  Generation 0 is the initial population: call it
 *                    with u = x and cost_u = cost(x).
 *   debye_de_run:    init, generation 0, then `iters` generations, each
 *                    [trial -> debye_fit_eval -> select]; with use_graph the
 *                    generation is captured once into a HIP graph and
 *                    replayed (bit-identical).  history needs
 *                    hist_ld >= iters + 1.  Calls with one plan must not overlap.
 * All pointers are device pointers; rows have stride ld >= max_poles.
 * ------------------------------------------------------------------------ */
typedef struct debye_de_params {
  double f_lo, f_hi, cr;   /* 0 <= f_lo <= f_hi <= 2, 0 <= cr <= 1 */
  uint64_t seed;
} debye_de_params;

int debye_de_init(const debye_batch *b, int64_t ld, const double *lb, const double *ub, debye_de_params p,
                  double *x, double *fit, double *best_cost, int64_t *best_idx, hipStream_t stream);
int debye_de_trial(const debye_batch *b, int64_t ld, const double *lb, const double *ub, debye_de_params p,
                   int32_t t, const double *x, double *u, hipStream_t stream);
int debye_de_select(const debye_batch *b, int64_t ld, int32_t t, const double *u, const double *cost_u, double *x,
                    double *fit, double *best_x, double *best_cost, int64_t *best_idx, double *history,
                    int64_t hist_ld, hipStream_t stream);

typedef struct debye_population {
  double *x, *u;          /* [n_cand][ld] members and trials */
  double *fit;            /* [n_cand] cost of the members */
  double *cost;           /* [n_cand] cost of the trials (workspace/output) */
  double *best_x;         /* [M][ld] */
  double *best_cost;      /* [M] */
  int64_t *best_idx;      /* [M] */
  double *history;        /* [M][hist_ld] or NULL */
  int64_t hist_ld;
  int8_t *status;         /* [n_cand] or NULL */
} debye_population;

int debye_de_run(const debye_plan *plan, const debye_batch *b, int64_t ld, const double *lb, const double *ub,
                 debye_de_params p, int32_t iters, double damping, uint32_t flags, const debye_population *pop,
                 int32_t use_graph, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Annealing (the paper's DA-DLS alternative, Sec. III-A; generalized
 * simulated annealing, Tsallis & Stariolo 1996, as in dual annealing),
 * batched: the candidates of material m are independent Markov chains over
 * log10 tau.  Generation t >= 1:
 *   visiting temperature   T(t) = t0 (2^(qv-1) - 1) / ((1 + t)^(qv-1) - 1)
 *   acceptance temperature Ta(t) = T(t) / t
 *   proposal  y = x + s(t) g (every coordinate), s(t) = T(t)^(1/(3-qv)) /
 *             sqrt(3 - qv), g_d Student-t with (3 - qv)/(qv - 1) degrees of
 *             freedom, wrapped periodically into [lb[m], ub[m]]
 *   accept    if cost(y) < cost(x); otherwise with probability
 *             [1 - (1 - qa)(cost(y) - cost(x))/Ta]^(1/(1-qa)) when positive
 *             (a NaN cost is never accepted)
 * then the material's best visited state (lowest index among equal costs)
 * if it improves; history[m * hist_ld + t] (may be NULL).  Random numbers:
 * Philox4x64-10, key (seed, material), counters listed in the library source;
 * exp and log are taken from their series, operation by operation, so that
 * runs are bit-identical to the CPU reference.  The state uses the
 * debye_population layout (x the chains, u the proposals, fit their costs).
 *   debye_da_init:   chains uniform in the box; fit, best_cost = +inf,
 *                    best_idx = -1.
 *   debye_da_visit:  y = proposals of generation t from x.
 *   debye_da_accept: generation t >= 1 as above; t = 0 takes y = x with
 *                    cost_y = cost(x) (the initial chains).
 *   debye_da_run:    init, generation 0, `iters` generations [visit ->
 *                    debye_fit_eval -> accept], optionally replayed from a
 *                    captured HIP graph (bit-identical); hist_ld >= iters + 1.
 * Defaults of the method: qv = 2.62, qa = -5, t0 = 5230.
 * ------------------------------------------------------------------------ */
typedef struct debye_da_params {
  double qv;      /* 1 < qv < 3 */
  double qa;      /* qa < 1 */
  double t0;      /* initial visiting temperature > 0 */
  uint64_t seed;
} debye_da_params;

int debye_da_init(const debye_batch *b, int64_t ld, const double *lb, const double *ub, debye_da_params p,
                  double *x, double *fit, double *best_cost, int64_t *best_idx, hipStream_t stream);
int debye_da_visit(const debye_batch *b, int64_t ld, const double *lb, const double *ub, debye_da_params p,
                   int32_t t, const double *x, double *y, hipStream_t stream);
int debye_da_accept(const debye_batch *b, int64_t ld, debye_da_params p, int32_t t, const double *y,
                    const double *cost_y, double *x, double *fit, double *best_x, double *best_cost,
                    int64_t *best_idx, double *history, int64_t hist_ld, hipStream_t stream);
int debye_da_run(const debye_plan *plan, const debye_batch *b, int64_t ld, const double *lb, const double *ub,
                 debye_da_params p, int32_t iters, double damping, uint32_t flags, const debye_population *pop,
                 int32_t use_graph, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Gradient polish: L-BFGS (Liu & Nocedal 1989; two-loop recursion, memory
 * `mem`), Armijo backtracking alpha = 1, 1/2, ... (max_trials, constant c1),
 * on one candidate per material, theta [M][ld] in place, inside the search box
 * [lb[m], ub[m]] (device [M]): every trial point is projected onto the box and
 * the sufficient-decrease test uses the projected displacement p,
 * C(trial) <= C + c1 min(g.p, 0) (no increase where clamping makes g.p
 * positive).  The first step (and any step whose quasi-Newton
 * direction is not a descent direction) is steepest descent scaled so that its
 * largest component is at most 1; a step with no acceptable trial leaves theta
 * unchanged; pairs with s.y <= 1e-300 are not stored (the history keeps its
 * older pairs).  The trials of a step are evaluated in three batched
 * launches: the full step (alpha = 1) of every material, the next four
 * halvings of the materials whose full step failed, and the remaining trials
 * of those still undecided (the result is the one a sequential halving search
 * returns).  A step with no acceptable trial leaves point, gradient and
 * history unchanged, so the material is left out of the later steps' launches
 * (its next steps would reject the same trials).
 *
 * The polish context owns every buffer (history, trials, gradients and the two
 * evaluation plans); debye_polish_create is the set-up call that allocates.
 * `shape` must describe one candidate per material (cand_off[m] = m); the
 * batches passed later must have the same shape.  The other calls only enqueue
 * work on `stream`: no allocation, no synchronisation, so a step can be
 * captured into a HIP graph.  Calls with one context must not overlap.
 *   debye_polish_begin:  cost and gradient at theta, history emptied.
 *   debye_polish_step:   one step (direction -> full steps -> further
 *                        trials where needed -> selection -> gradient at the
 *                        accepted point -> history update);
 *                        cost_hist [M][steps+1] (may be NULL) receives the cost
 *                        before step `step` and, at step == steps-1, the cost
 *                        at the end.
 *   debye_lbfgs_polish:  begin, then steps 0 .. p.steps-1 (cost_hist as above,
 *                        non-increasing along each row).
 * ------------------------------------------------------------------------ */
typedef struct debye_lbfgs_params {
  int32_t steps, mem, max_trials;
  double c1;
} debye_lbfgs_params;

typedef struct debye_polish debye_polish;

int debye_polish_create(const debye_batch *shape, const int64_t *f_off_host, const int32_t *n_poles_host, int64_t ld,
                        debye_lbfgs_params p, debye_polish **out);
int debye_polish_destroy(debye_polish *polish);
int debye_polish_begin(debye_polish *polish, const debye_batch *b, const double *theta, double damping,
                       uint32_t flags, hipStream_t stream);
int debye_polish_step(debye_polish *polish, const debye_batch *b, double *theta, const double *lb, const double *ub,
                      double damping, uint32_t flags, int32_t step, double *cost_hist, hipStream_t stream);
int debye_lbfgs_polish(debye_polish *polish, const debye_batch *b, double *theta, const double *lb, const double *ub,
                       double damping, uint32_t flags, double *cost_hist, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* DEBYEFIT_H */
