/*
 * pgvimp.h - C ABI of the MI355X (gfx950) P-GVIMP hot-path library.
 *
 * P-GVIMP (arXiv 2411.03416) plans a Gaussian trajectory distribution
 * N(mu, Lambda^-1) over N support states x_0..x_{N-1} (each n-dim) of a
 * linear time-varying SDE dX = (A_t X + a_t) dt + B_t dW (Sec. 2.2, eq.
 * dynamics_linear) by a KL-proximal iteration (Theorem 1, Alg. 1).  One
 * iteration of the hot path is:
 *   - marginals Sigma_ii, Sigma_{i,i+1} of the block-tridiagonal precision
 *     by Gaussian belief propagation on the chain (Sec. 5.1);
 *   - per-state Gauss-Hermite expectations of the hinge signed-distance
 *     collision cost in the derivative-free Stein form (Sec. 4.1 eq.
 *     gradients_psid, Sec. 4.3 eq. GH_quadrature_matmul) and closed-form
 *     expectations of the GP-prior factors;
 *   - the precision/mean update of Theorem 1 (eq. mu_Sigma_update) with the
 *     step size chosen by halving until the new precision is positive
 *     definite and KL(q_{k+1} || q_k) <= kl_bound (Alg. 1, App. C).
 * Nonlinear drifts are handled by statistical linear regression (Sec. 6.2,
 * Alg. 2) before each run of the iteration.
 *
 * Conventions
 *   - All matrices are row-major FP64.  Block arrays are [count][n][n].
 *     The precision is given by its diagonal blocks D_i = Lambda_{i,i}
 *     (N blocks) and super-diagonal blocks U_i = Lambda_{i,i+1} (N-1 blocks);
 *     covariances likewise (Sigma_{i,i}, Sigma_{i,i+1}).
 *   - Unless a function says otherwise, array arguments are HOST pointers
 *     owned by the caller.  With pgvimp_engine_cfg.io_on_device = 1 the
 *     output arrays of pgvimp_marginals, pgvimp_factor_expectations,
 *     pgvimp_get_state and pgvimp_slr_linearize are DEVICE pointers instead
 *     and are written asynchronously on the context's stream.
 *   - No pointer passed in is retained after the call returns; inputs are
 *     copied to device memory owned by the context.
 *   - Every function returns 0 (PGVIMP_OK) or a negative error code.  The
 *     message of the last failure is available from pgvimp_last_error.  A
 *     failure in one plan never modifies another plan's state.
 */
#ifndef PGVIMP_H
#define PGVIMP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define PGVIMP_OK 0
#define PGVIMP_EINVAL (-1)  /* null pointer, bad size, non-finite input    */
#define PGVIMP_ENOMEM (-2)  /* device memory or context capacity exhausted */
#define PGVIMP_ENOTPD (-3)  /* a precision/covariance is not positive def. */
#define PGVIMP_ENOCONV (-4) /* no step size passed the rule (plan unchanged)*/
#define PGVIMP_EDEVICE (-5) /* HIP runtime error or library not usable     */
#define PGVIMP_EBUSY (-6)   /* no free plan slot                           */

/* precision modes */
#define PGVIMP_FP64 0  /* every step in FP64                                   */
#define PGVIMP_MIXED 1 /* quadrature nodes, SDF lookups, forward kinematics and
                          the cost in FP32; Cholesky, triangular solves, GBP,
                          the update and the linearisation in FP64            */

/* collision models (which configuration a state's collision factor sees) */
#define PGVIMP_COLL_NONE 0    /* no collision factor                          */
#define PGVIMP_COLL_POINT2D 1 /* point at (x[ci0], x[ci1]), bilinear 2-D SDF  */
#define PGVIMP_COLL_POINT3D 2 /* point at x[ci0..2], trilinear 3-D SDF        */
#define PGVIMP_COLL_ARM3D 3   /* 7 joint angles x[ci0..6] -> forward kinematics
                                 of a serial chain -> spheres, trilinear SDF  */

/* update rules of one iteration */
#define PGVIMP_UPDATE_PROX 0 /* KL-proximal step of Theorem 1 (eq.
                                mu_Sigma_update)                             */
#define PGVIMP_UPDATE_NGD 1  /* natural-gradient step (Sec. 3.1(d), eq.
                                ngd_proximal): descent on J = E[psi] - T H(q)
                                in the natural parameters,
                                Lambda' = Lambda_k + beta (K^-1 + H - T Lambda_k),
                                Lambda' (mu' - mu_k) = -beta (K^-1 mu_k - eta + g) */

/* quadrature rules of the collision expectations */
#define PGVIMP_QUAD_TENSOR 0 /* tensor Gauss-Hermite, p points per axis       */
#define PGVIMP_QUAD_SPARSE 1 /* Smolyak combination of Gauss-Hermite tensor
                                rules of level k (at most 65536 nodes)       */

/* nonlinear models for pgvimp_slr_linearize */
#define PGVIMP_MODEL_QUAD2D 1 /* planar quadrotor drift of Sec. 7.3 eq.
                                 planar_quad with u = 0; state (x, z, phi,
                                 vx, vz, phidot); model_params = {gravity}   */

#define PGVIMP_MAX_COLL_DIM 8
#define PGVIMP_MAX_SPHERES 32
#define PGVIMP_ARM_DOF 7

typedef struct pgvimp_ctx pgvimp_ctx;

/*
 * One planning problem (Alg. 1 inputs).  All pointers are host pointers,
 * read during the call that receives the struct.
 *
 * Dynamics: if ltv == 0, A [n*n], a [n], B [n*m] hold for every interval;
 * if ltv == 1 they are [N-1][n][n], [N-1][n], [N-1][n][m], interval i being
 * [t_i, t_{i+1}).  Qc [m*m] is the noise spectral density (SPD).  The
 * start and goal factors are N(x_0; mu_start, Sig_start) and
 * N(x_{N-1}; mu_goal, Sig_goal) (SPD covariances).
 *
 * Iteration: temperature T > 0 weights the entropy in E[psi] - T H(q);
 * the step size starts at beta_max > 0 and is halved at most max_bisect
 * times (1 <= max_bisect <= 64); kl_bound > 0 (may be +inf) bounds KL(q_{k+1} || q_k); n_iters is
 * the plan's iteration budget consumed by pgvimp_prox_step.
 *
 * Collision cost of state x: psi = obs_weight * sum_s max(0, hinge_eps +
 * r_s - sdf(c_s(x)))^2, where c_s are the collision points (the point
 * itself, or forward-kinematics spheres) and r_s their radii.  The SDF is
 * an FP32 grid sampled at nodes origin + (ix, iy, iz) * cell, stored
 * sdf[iy][ix] (2-D, gz = 1) or sdf[iz][iy][ix] (3-D); lookups are bilinear
 * or trilinear with clamping to the grid.  The library keeps the grid and a
 * table of its cell corners (16 bytes a cell) on the device, which must stay
 * under 2 GiB ((gx-1)(gy-1)gz * 16 bytes; larger grids are rejected with
 * PGVIMP_EINVAL).  Plans of one context whose grids are identical (same
 * dimensions and values) share one device copy.  gh_points p in [1, 10] points per
 * configuration dimension (tensor rule, p^d nodes).  coll_states: 0 = every
 * support state carries a collision factor, 1 = only interior states.
 *
 * Arm forward kinematics (PGVIMP_COLL_ARM3D): joint k rotates about its
 * local axis fk_axes[k] (0 = x, 1 = y, 2 = z) and link k then extends by
 * fk_link_len[k] along the rotated local z; frame 0 starts at fk_base [3].
 * Sphere s sits on link fk_sphere_link[s] at fraction fk_sphere_frac[s] of
 * its length.
 */
typedef struct pgvimp_problem {
    int32_t n, m, N;
    double dt;
    int32_t ltv;
    const double *A, *a, *B, *Qc;
    const double *mu_start, *Sig_start, *mu_goal, *Sig_goal;
    double temperature, beta_max, kl_bound;
    int32_t max_bisect, n_iters;
    int32_t coll_kind, coll_dim;
    int32_t coll_index[PGVIMP_MAX_COLL_DIM];
    int32_t gh_points, coll_states;
    const float *sdf;
    int32_t gx, gy, gz;
    double origin[3];
    double cell, hinge_eps, obs_weight;
    int32_t n_spheres;
    const double *sphere_radius;
    const double *fk_base, *fk_link_len, *fk_sphere_frac;
    const int32_t *fk_axes, *fk_sphere_link;
    const double *mu_init; /* optional [N][n] initial mean; NULL -> prior mean */
    int32_t segments;      /* chain segments for this plan (0 = context default) */
    int32_t expect_group;  /* factors per expectation workgroup: 32, 64, 128,
                              256 or 0 = chosen per launch (speed only)   */
    int32_t quadrature;    /* PGVIMP_QUAD_TENSOR: gh_points = p points per
                              axis (p^d nodes); PGVIMP_QUAD_SPARSE: Smolyak
                              sparse grid of level k = gh_points (Sec. 4.3
                              Lemma 1), exact to total degree 2k - 1      */
    int32_t update;        /* PGVIMP_UPDATE_PROX or PGVIMP_UPDATE_NGD; both
                              use the same step-size rule (halving from
                              beta_max until Lambda' is positive definite
                              and KL(q' || q_k) <= kl_bound)              */
} pgvimp_problem;

/*
 * Engine (context) configuration.  A context holds up to max_plans plans of
 * one state dimension n with at most max_states support states in total,
 * resident on one device, plus a heap of heap_bytes for maps and per-plan
 * model data.  precision is PGVIMP_FP64 or PGVIMP_MIXED.  stream is a
 * hipStream_t on which all work is enqueued (NULL = a non-blocking stream of
 * default priority created and owned by the context).  If
 * dev_arena is non-NULL the context sub-allocates all its device memory
 * from that caller-owned buffer of arena_bytes bytes (which must outlive
 * the context); otherwise it allocates its own.  segments overrides the
 * tuned chain segments (0 = tuned default); expect_group fixes the factors
 * per workgroup of the expectation kernel (32, 64, 128 or 256; 0 = the
 * largest that gives every compute unit four workgroups; the arm uses 32,
 * or with 0 also 8 when 32 would give fewer than two workgroups per compute
 * unit; speed only, never results);
 * use_graph = 1 captures pgvimp_prox_step's iterations in a HIP graph sized
 * to the plans present (re-captured when they change); use_graph = 2 sizes
 * the graph to the full capacity so plans can join and leave without a new
 * capture (serving).
 * Step sizes of the halving sequence (Alg. 1) are evaluated concurrently
 * in windows: each window of a plan continues where its previous one ended,
 * until one holds a passing step.  A window's width is the number of
 * compute units divided by the number of plans still searching, clamped to
 * [trial_width, trial_slots]: trial_width (0 = 8 for n <= 4, 24 for
 * n >= 6, at most 64) is the narrowest window, trial_slots (0 = 2 *
 * trial_width for n <= 4, trial_width for n >= 6; at least trial_width, at
 * most 64) the widest, and the trial scratch scales with trial_slots.  (For
 * n >= 6 one trial is a long chain of small latency-bound block steps, so
 * several trials per compute unit in one wide window beat narrow windows
 * run one after another.)  trial_lookahead > 0 cuts each plan's first window of an
 * iteration to t + trial_lookahead step sizes (at least 1), t = the number
 * its previous iteration tried; 0 = no cut.  All three change speed and
 * memory, never results: the accepted step is the first passing one in
 * halving order whatever the windows.
 */
typedef struct pgvimp_engine_cfg {
    int32_t device, n, precision, max_plans;
    int64_t max_states, heap_bytes;
    void *stream;
    void *dev_arena;
    uint64_t arena_bytes;
    int32_t io_on_device, segments, expect_group, use_graph;
    int32_t trial_width, trial_lookahead, trial_slots;
} pgvimp_engine_cfg;

/*
 * Per-plan statistics of the last iteration run by pgvimp_prox_step.  The
 * cost breakdown describes q_k, the iterate the iteration started from
 * (Sec. 2.2: J(q) = E[psi] - T H(q), psi = prior factors + collision
 * factors): total_cost = E_prior + E_coll + entropy_cost with entropy_cost =
 * -T H(q_k), T the plan's temperature during the iteration.  logdet and
 * entropy describe q_{k+1}.
 */
typedef struct pgvimp_stats {
    double beta;    /* accepted step size (0 if none)                       */
    double kl;      /* KL(q_{k+1} || q_k) of the accepted step              */
    double E_coll;  /* sum of collision-factor expectations at q_k          */
    double E_prior; /* sum of prior-factor expectations at q_k              */
    double logdet;  /* log det of the precision after the iteration         */
    double entropy; /* entropy of q after the iteration                     */
    double temperature;  /* T of the iteration                              */
    double entropy_cost; /* -T H(q_k)                                       */
    double total_cost;   /* E_prior + E_coll - T H(q_k) = J(q_k)            */
    int32_t status; /* 0, PGVIMP_ENOTPD (input) or PGVIMP_ENOCONV           */
    int32_t trials; /* step sizes tried in the last iteration               */
    int32_t iters_done, iters_left;
    int32_t trials_total; /* step sizes tried since the plan was (re)started  */
    int32_t evals_total;  /* step sizes evaluated since then, counting the
                             speculative ones of each window (>= trials_total) */
} pgvimp_stats;

/*
 * Create a context and add n_probs plans (plan ids 0..n_probs-1).  For each
 * plan the GP prior is built on the device (Alg. 1: transition kernels,
 * Grammians, K^-1 and the prior mean), the state is initialised to
 * mu_0 = prior mean (or mu_init) and Lambda_0 = K^-1, and its marginals are
 * computed.  Returns EINVAL for invalid problems/config, ENOMEM if the
 * plans do not fit, EDEVICE for HIP failures.  *out is NULL on failure.
 */
int pgvimp_create(const pgvimp_problem *probs, int32_t n_probs, const pgvimp_engine_cfg *cfg,
                  pgvimp_ctx **out);

/* Release the context and all device memory it allocated. */
int pgvimp_destroy(pgvimp_ctx *ctx);

/*
 * Add one plan to a live context (serving admission).  *plan_out receives
 * the slot id.  EBUSY if no slot is free, ENOMEM if its states or map do not
 * fit in the remaining capacity; the context is unchanged on failure.
 */
int pgvimp_add_plan(pgvimp_ctx *ctx, const pgvimp_problem *prob, int32_t *plan_out);

/* Free a plan's slot, states and heap memory. */
int pgvimp_remove_plan(pgvimp_ctx *ctx, int32_t plan);

/*
 * Marginal covariances of the plan's current precision by GBP on the chain
 * (Sec. 5.1, eqs. messages and belief_lambda): cov_diag [N][n][n] =
 * Sigma_{i,i}, cov_off [N-1][n][n] = Sigma_{i,i+1}, *logdet = log det
 * Lambda.  Any output pointer may be NULL.  ENOTPD if Lambda is not
 * positive definite.
 */
int pgvimp_marginals(pgvimp_ctx *ctx, int32_t plan, double *cov_diag, double *cov_off, double *logdet);

/*
 * Evaluate the collision-factor expectations (Sec. 4.1 eq. gradients_psid,
 * Sec. 4.3) of every live plan at its current mean and marginals, reps >= 1
 * times, leaving them on the device (no readback; the results are the ones
 * the next iteration would use).  With pgvimp_profile enabled each launch is
 * timed (kind PGVIMP_K_EXPECT of pgvimp_kernel_times).  Meant for measuring
 * the expectation stage alone.  Errors: EINVAL (bad reps), EDEVICE.
 */
int pgvimp_expect_all(pgvimp_ctx *ctx, int32_t reps);

/*
 * Per-factor expectations at the plan's current (mu, marginals):
 * E_coll [N] = E[psi_i]; grad [N][n] = Sigma_i^-1 E[(x - mu_i) psi_i];
 * hess [N][n][n] = 2 grad_Sigma = Sigma_i^-1 (E[(x-mu)(x-mu)^T psi] -
 * E[psi] Sigma_i) Sigma_i^-1 (Sec. 4.1 eq. gradients_psid), embedded with
 * zeros outside the configuration coordinates; E_prior [N+1] = closed-form
 * expected prior factor costs 1/2 E[r^T W r] ordered (start, transitions
 * 0..N-2, goal).  Any output pointer may be NULL.
 */
int pgvimp_factor_expectations(pgvimp_ctx *ctx, int32_t plan, double *E_coll, double *grad,
                               double *hess, double *E_prior);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * outputs as pgvimp_factor_expectations, but host outputs are staged through
 * a fixed library array of 4 MiB per device (2^19 doubles) instead of a
 * buffer allocated on first use, and the call makes no device allocation or
 * free.  The array's device address is looked up once per device when the
 * first context on it is created.  ENOMEM if the largest output
 * (max(N*n*n, N+1) doubles) exceeds the array (host outputs only; with
 * io_on_device = 1 nothing is staged).  Every call on one device shares that
 * device's array: calls that overlap on one device (from several threads or
 * contexts) race and must be serialised by the caller.  The call
 * synchronises the context's stream before it returns.
 */
int pgvimp_factor_expectations_noalloc(pgvimp_ctx *ctx, int32_t plan, double *E_coll, double *grad,
                                       double *hess, double *E_prior);

/*
 * Run n_iters KL-proximal iterations (Alg. 1) on every live plan that has
 * budget left: expectations, step-size selection, update (Theorem 1), new
 * marginals.  per_plan (host, may be NULL) receives max_plans entries;
 * entries of empty slots are zeroed.  A plan whose step rule fails keeps
 * its state and reports status ENOCONV; the call still returns 0.
 */
int pgvimp_prox_step(pgvimp_ctx *ctx, int32_t n_iters, pgvimp_stats *per_plan);

/*
 * Solve every live plan from scratch: rebuild its prior from its stored
 * dynamics (Alg. 1 set-up), reset mu_0 = prior mean, Lambda_0 = K^-1 and
 * its marginals and its iteration budget, then run n_iters iterations as in
 * pgvimp_prox_step.  With use_graph the whole sequence is one HIP graph.
 */
int pgvimp_solve(pgvimp_ctx *ctx, int32_t n_iters, pgvimp_stats *per_plan);

/*
 * Statistical linear regression (Sec. 6.2, eqs. SLR_best_ai and
 * SLR_best_Ai) of the model's drift about every support state's current
 * marginal N(mu_i, Sigma_ii), with a gh_points^n tensor Gauss-Hermite rule:
 * A_out [N][n][n], a_out [N][n] (either may be NULL).  If rebuild_prior is
 * non-zero the plan's prior is rebuilt from (A_i, a_i) held on
 * [t_i, t_{i+1}) with the plan's B and Qc, the precision restarts from the
 * new K^-1, the mean is kept, and the marginals are recomputed (Alg. 2).
 */
int pgvimp_slr_linearize(pgvimp_ctx *ctx, int32_t plan, int32_t model, const double *model_params,
                         int32_t gh_points, int32_t rebuild_prior, double *A_out, double *a_out);

/*
 * One round of Alg. 2 (i-P-GVIMP): statistical linearisation of the model's
 * drift (Sec. 6.2, as pgvimp_slr_linearize with rebuild_prior = 1), then the
 * plan's iteration budget is set to n_iters, so the next pgvimp_prox_step
 * calls run the round's P-GVIMP iterations (Alg. 1) on the rebuilt LTV
 * prior.  The first round passes the nominal trajectory: nominal_mean
 * [N][n] and per-state covariances nominal_cov [N][n][n] (host, SPD); they
 * become the plan's mean and marginals before the regression, and the mean
 * is kept when the precision restarts from the new K^-1.  Later rounds pass
 * NULL for both and linearise about the plan's current marginals.  A_out
 * and a_out as in pgvimp_slr_linearize (either may be NULL).  Errors: EINVAL
 * (only one of the nominal arrays given, a non-finite value, a covariance
 * block that is not SPD, n_iters < 0, a model the context's n does not
 * fit; the plan is unchanged), ENOTPD (the linearised prior is not positive
 * definite), EDEVICE.
 */
int pgvimp_slr_round(pgvimp_ctx *ctx, int32_t plan, int32_t model, const double *model_params,
                     int32_t gh_points, const double *nominal_mean, const double *nominal_cov,
                     int32_t n_iters, double *A_out, double *a_out);

/*
 * A later round of Alg. 2 for n_plans plans at once (plans [n_plans],
 * distinct live plan indices): for each, the drift's statistical
 * linearisation about its current marginals (Sec. 6.2), then the LTV
 * priors of all of them are rebuilt, their precisions restart from the new
 * K^-1 (means kept) and their marginals are recomputed in shared launches;
 * each plan's budget becomes n_iters.  The other live plans are untouched.
 * status [n_plans] (host, may be NULL) receives PGVIMP_OK or PGVIMP_ENOTPD
 * per plan: a plan whose linearised prior is not positive definite gets a
 * budget of 0 instead of failing the call.  The same results as
 * pgvimp_slr_round on each plan in turn.  Errors: EINVAL (bad arguments:
 * a plan listed twice or not live, n_iters < 0, a model the context's n
 * does not fit; nothing is changed), EDEVICE.
 */
int pgvimp_slr_round_many(pgvimp_ctx *ctx, int32_t n_plans, const int32_t *plans, int32_t model,
                          const double *model_params, int32_t gh_points, int32_t n_iters, int32_t *status);

/* Read the plan's mean [N][n] and precision blocks D [N][n][n], U [N-1][n][n]. */
int pgvimp_get_state(pgvimp_ctx *ctx, int32_t plan, double *mu, double *prec_diag, double *prec_off);

/*
 * Overwrite the plan's mean and precision (host arrays as in get_state) and
 * recompute its marginals.  ENOTPD (state unchanged) if the precision is
 * not positive definite.  Any of the three may be NULL to keep that part.
 */
int pgvimp_set_state(pgvimp_ctx *ctx, int32_t plan, const double *mu, const double *prec_diag,
                     const double *prec_off);

/* Set the plan's remaining iteration budget. */
int pgvimp_set_budget(pgvimp_ctx *ctx, int32_t plan, int32_t iters_left);

/*
 * Set the plan's temperature T > 0 (the weight of the entropy in the
 * objective E[psi] - T H(q), Sec. 2.2) for the iterations that follow: the
 * paper's runs use a low temperature until the plan is collision-free, then
 * a high one that emphasises the entropy (Sec. 7).  Takes effect on the
 * next pgvimp_prox_step, also inside a captured graph.  EINVAL for T <= 0 or
 * not finite (the plan is unchanged).
 */
int pgvimp_set_temperature(pgvimp_ctx *ctx, int32_t plan, double temperature);

/* Change the stream used by the context (hipStream_t; NULL = a new stream
 * owned by the context).  Waits for the old stream first. */
int pgvimp_set_stream(pgvimp_ctx *ctx, void *stream);

/* Block until all work enqueued by the context has finished. */
int pgvimp_sync(pgvimp_ctx *ctx);

/*
 * Launch shapes in use: *segments = chain segments of the first live plan of
 * N states (the context default for N if there is none), *group = factors
 * per workgroup of the expectation kernel for the live plans (of the first
 * live plan's request).  Either pointer may be NULL.
 */
int pgvimp_launch_shape(pgvimp_ctx *ctx, int32_t N, int32_t *segments, int32_t *group);

/* kernel kinds reported by pgvimp_kernel_times */
#define PGVIMP_K_EXPECT 0  /* collision-factor expectations                */
#define PGVIMP_K_PREP 1    /* per-iteration set-up (K^-1 + H, rhs, costs)  */
#define PGVIMP_K_TRIAL 2   /* a window of trial step sizes (GBP + solve)   */
#define PGVIMP_K_SELECT 3  /* pick the first passing step, write back      */
#define PGVIMP_K_RESTART 4 /* prior build + initial state (pgvimp_solve)   */
#define PGVIMP_NKERNELS 5

/*
 * Kernel timing.  pgvimp_profile(ctx, 1) makes pgvimp_prox_step and
 * pgvimp_solve launch their kernels directly (not through a HIP graph: events
 * recorded inside a captured graph cannot be timed) with a HIP event pair on
 * the context's stream around every launch.  pgvimp_kernel_times fills
 * mean_ms[PGVIMP_NKERNELS] (mean duration per launch, milliseconds) and
 * launches[PGVIMP_NKERNELS] over the launches timed since the last call with
 * reset = 1; either pointer may be NULL.
 */
int pgvimp_profile(pgvimp_ctx *ctx, int32_t enable);
int pgvimp_kernel_times(pgvimp_ctx *ctx, int32_t reset, double *mean_ms, int64_t *launches);

/* Bytes of device memory held by the context. */
int64_t pgvimp_device_bytes(const pgvimp_ctx *ctx);

/*
 * Bytes of device memory a context created with cfg needs (the size of the
 * caller-provided arena, cfg->dev_arena), or a negative error code.
 */
int64_t pgvimp_arena_bytes(const pgvimp_engine_cfg *cfg);

/*
 * Bytes of context heap (cfg->heap_bytes) one plan of this problem takes:
 * its SDF grid (shared with live plans of the same grid in a context) and
 * its model data (dynamics, factors, forward kinematics, sparse rule).
 * Negative error code for an invalid problem.
 */
int64_t pgvimp_plan_heap_bytes(const pgvimp_problem *prob);

/* Message of the last failure on this context (or of create if ctx NULL). */
const char *pgvimp_last_error(const pgvimp_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* PGVIMP_H */
