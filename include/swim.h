/*
 * swim.h -- C ABI of libswim: a batched forward model of elastic filament
 * swimmers in a Brinkman fluid, and the approximate-Bayesian (ABC) machinery
 * around it, on AMD Instinct MI355X (gfx950).
 *
 * Method (Larson, Olson & Matzavinos, "Bayesian uncertainty quantification for
 * micro-swimmers with fully resolved hydrodynamics"):
 *   - the flagellum is N Lagrangian points X_k, k = 0..N-1, of a filament of
 *     length 1 (ds = 1/(N-1)), initially straight along x from (x0, y0);
 *   - forces F = -dE/dX (eq. Fenergy) of the discrete tensile energy
 *     E_t = S_s sum_k (|X_{k+1}-X_k|/ds - 1)^2 ds (eq. EFT, Hookean springs)
 *     and bending energy E_b = S_b sum_{k=1}^{N-2} (kappa_k - kappa0_k)^2 ds
 *     (eq. EFB), kappa from eq. (curva) with centred differences, and the
 *     preferred curvature kappa0(s,t) = -k^2 b sin(k s - omega t + phase)
 *     (second derivative of the Appendix beat, untapered);
 *   - velocities from the regularized Brinkmanlet sum of eq. (BrV), Sec. 2.1,
 *     over all points of a system (all its swimmers), blob width
 *     eps = eps_over_ds * ds, resistance alpha (alpha = 0: Stokes limit);
 *   - no-slip update dX/dt = v(X) by forward Euler (Sec. 2.1, Appendix).
 *
 * Conventions
 *   - Every call returns SWIM_OK (0) or a negative error code and never throws;
 *     swim_last_error() returns a thread-local message for the last error.
 *   - "device" pointers are HIP device memory owned by the caller (e.g. torch
 *     tensors); "host" pointers are ordinary host memory.  The library never
 *     frees caller memory; a context owns only its own workspace.
 *   - dtype selects the arithmetic: SWIM_F32 (float) or SWIM_F64 (double) --
 *     the same kernel source instantiated twice.  Arrays typed "void*" hold
 *     float or double accordingly.
 *   - Calls taking a stream are asynchronous on that hipStream_t (NULL = the
 *     context's stream); calls documented as synchronous wait for their work.
 *     The context's workspace is shared by all its calls: a call on another
 *     stream than the previous call first makes its stream wait for the work
 *     enqueued on that previous stream (so keep a stream alive until a later
 *     call has run on another one).
 *   - A context is not thread-safe: use one per host thread.
 *   - Per-sample numerical failure (blow-up of the explicit scheme) is a
 *     status value, not an error.
 */
#ifndef SWIM_H
#define SWIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SWIM_OK 0
#define SWIM_EINVAL (-1)  /* bad argument; nothing was launched      */
#define SWIM_EHIP (-2)    /* a HIP runtime call failed               */
#define SWIM_ENOMEM (-3)  /* device or pinned allocation failed      */
#define SWIM_ESTATE (-4)  /* context unusable (e.g. after a HIP error) */

#define SWIM_F32 0
#define SWIM_F64 1

#define SWIM_ST_OK 0        /* run completed                          */
#define SWIM_ST_NONFINITE 1 /* a position became NaN/Inf; run stopped */
#define SWIM_ST_BOUND 2     /* |x| or |y| exceeded 1e3; run stopped   */
#define SWIM_ST_BADPARAM 3  /* parameters outside the domain (alpha < 0,
                               alpha*eps > 1, non-finite); not run     */
#define SWIM_ST_REJECTED 4  /* abc_prescreened only: the run stopped once its head's
                               running squared deviation from the data passed the
                               tolerance (its distance exceeds it)              */

/* Parameter row of one filament: 9 doubles in this order. */
#define SWIM_P_ALPHA 0 /* Brinkman resistance alpha >= 0 (one value per system)  */
#define SWIM_P_SB 1    /* bending stiffness S_b (K_C of eq. EFB)                  */
#define SWIM_P_SS 2    /* stretching stiffness S_s (K_T of eq. EFT)               */
#define SWIM_P_B 3     /* beat amplitude b                                        */
#define SWIM_P_OMEGA 4 /* beat angular frequency omega                            */
#define SWIM_P_K 5     /* beat wavenumber k                                       */
#define SWIM_P_PHASE 6 /* beat phase                                              */
#define SWIM_P_X0 7    /* start point x0 of the filament                          */
#define SWIM_P_Y0 8    /* start point y0                                          */
#define SWIM_NPARAM 9

typedef struct swim_ctx swim_ctx;

/* Creates a context on HIP device `device` with its own stream (a blocking
 * stream at the default priority: it is ordered with work on the legacy NULL
 * stream, so host-side preparation of buffers on that stream needs no extra
 * synchronization).  *out is set to NULL on failure. */
int swim_create(swim_ctx **out, int device);
void swim_destroy(swim_ctx *ctx);
const char *swim_last_error(void);
int swim_version(void);

/* Launch options of a context (the autotuner sets the first two):
 *   SWIM_OPT_WPS     wavefronts that share one system in the persistent
 *                    kernel, splitting its pair work: 0 (automatic: the
 *                    autotuned value, else 8 for FP32 systems of 65..128
 *                    points and 16 otherwise), 1, 2, 4, 8, 16 (reduced
 *                    when the partial sums would not fit LDS).  Systems above 256 points need at least 2: a
 *                    forward call with 1 and such a system fails with
 *                    SWIM_EINVAL (the automatic choice never takes 1 there);
 *   SWIM_OPT_BIG_TPL the large-system step (systems above 512 points):
 *                    0 (automatic: FP32 takes the symmetric step, every
 *                    pair evaluated once for both points, in tile pairs of
 *                    256 points with a partial-sum buffer reduced in a
 *                    fixed order; FP64 the one-sided kernel at one target
 *                    per lane), or 1, 2, 4: the one-sided kernel at that
 *                    many targets per lane;
 *   SWIM_OPT_GRAPH   forward runs as a captured hipGraph: 0 never (eager
 *                    launches), 1 (default) capture when a call repeats the
 *                    previous call's layout (systems, sizes, run length,
 *                    options and every buffer address) and replay it while
 *                    that layout recurs, 2 capture every new layout at once.
 *                    Parameter values may change between replays: they are
 *                    uploaded before the graph runs.
 *   SWIM_OPT_BLOB    the regularization blob of the velocity kernel:
 *                    SWIM_BLOB_PAPER (default), the blob of eq. (eqnblob),
 *                    or SWIM_BLOB_READING, the unit-mass blob
 *                    c eps^2/(2 pi) [alpha^2 K0(alpha R)/R^2 + 2 alpha
 *                    K1(alpha R)/R^3] (eps^2/(pi R^4) at alpha = 0), whose
 *                    Brinkmanlet has a closed form for every alpha.  The
 *                    paper's blob has a closed form in the Stokes limit,
 *                    H2 = (R + 2 eps)/(4 pi R (R + eps)^2) and
 *                    H1 = -[ln(R + eps) - eps (R + 2 eps)/(R (R + eps))]/(4 pi)
 *                    - 1/(8 pi).  For alpha > 0 there is none: g, the
 *                    solution of (Delta - alpha^2) g = phi, comes from two
 *                    radial integrals of the blob against I0 and K0 (Graf's
 *                    addition theorem), taken by FP64 Gauss-Legendre
 *                    quadrature, with H1 = M/r^2 - g, H2 = (g - 2M/r^2)/r^2,
 *                    M = int_0^r s g ds, and g(0) in closed form from the
 *                    sine and cosine integrals.  FP32 runs read it from the
 *                    per-system tables, built once per launch by one sweep
 *                    over the table's 2113 nodes in increasing r (prefix
 *                    and suffix sums of the two integrals over the gaps
 *                    between nodes, a far-field expansion beyond
 *                    alpha r = 40); FP64
 *                    evaluates the quadrature per pair, a few hundred
 *                    times the cost of the closed forms (a reference mode
 *                    for small systems).  It applies to every velocity and
 *                    pressure evaluation, including the pressure's blob
 *                    mass (1 - eps^3/R^3).
 * Read-only counters (swim_get_option): SWIM_OPT_GRAPH_LAUNCHES (graph
 * replays and first launches so far), SWIM_OPT_GRAPH_CAPTURES.
 * SWIM_OPT_TIME_KERNEL = 1 makes every forward call (swim_forward and the
 * calls that run it) launch eagerly and record two timing events on its
 * stream, right before and right after its persistent launches (the
 * per-system set-up excluded; several size buckets: from before their fork
 * to after their join; a chunked call: its last chunk); SWIM_OPT_KERNEL_US
 * (read-only) then waits for the last such call and returns that interval
 * in microseconds (SWIM_ESTATE if no timed call was made since the option
 * was set).
 * Results do not depend on the launch options beyond rounding of the
 * source-split partial sums.  SWIM_EINVAL for an unknown key or value. */
#define SWIM_OPT_WPS 1
#define SWIM_OPT_BIG_TPL 2
#define SWIM_OPT_GRAPH 3
#define SWIM_OPT_GRAPH_LAUNCHES 4
#define SWIM_OPT_GRAPH_CAPTURES 5
#define SWIM_OPT_BLOB 6
#define SWIM_OPT_EARLY_STOP 7 /* abc_prescreened's early stop of rejected re-runs: 1 (default) or 0 */
#define SWIM_OPT_TIME_KERNEL 8 /* 1: time the persistent launches of forward calls (default 0) */
#define SWIM_OPT_KERNEL_US 9   /* read-only: microseconds of the last timed forward call's launches */
#define SWIM_BLOB_READING 0 /* the unit-mass blob whose Brinkmanlet has a closed form for all alpha */
#define SWIM_BLOB_PAPER 1   /* default: eq. (eqnblob), 3 eps^3 / (2 pi (r^2 + eps^2)^(5/2)) */
int swim_set_option(swim_ctx *ctx, int32_t key, int32_t value);
int swim_get_option(swim_ctx *ctx, int32_t key, int32_t *value);

/* Autotuner of the launch shapes (synchronous).  Times forward runs of
 * probe_steps steps of the given batch (layout and parameter rows as for
 * swim_forward; params device) on the context's stream, eagerly:
 *   - for every size bucket of the persistent kernel the forward calls
 *     launch for this batch (systems of up to 64*tpl points, tpl in
 *     {1,2,3,4,6,8}, after the merging that swim_forward describes), the
 *     waves per system among 2, 4, 8, 16 (those whose partial sums fit the
 *     LDS), each bucket probed alone on its systems of the batch (the
 *     buckets of a call run side by side, so the call's time does not see
 *     a bucket off its longest path): the most waves whose probe is within
 *     5 % of the fastest (a run's own speed grows with its waves, and the
 *     longest runs bound a launch's time, which a short probe does not
 *     show).  The probes copy params to the host and allocate a device
 *     buffer of the same size;
 *   - if the batch has systems over 512 points, the large-system step:
 *     the one-sided kernel at 1, 2, 4 targets per lane and, for FP32, the
 *     symmetric step (SWIM_OPT_BIG_TPL = 0).
 * The choices stay in the context (used by every later run whose
 * SWIM_OPT_WPS is 0; the large-system choice sets SWIM_OPT_BIG_TPL) and
 * are returned in chosen (host int32[9]: waves per system for tpl = 1..8,
 * 0 where not tuned, then the large-system choice, SWIM_OPT_BIG_TPL's
 * value). */
int swim_autotune(swim_ctx *ctx, int32_t dtype, int64_t n_sys, const int32_t *N,
                  const int32_t *n_swim, const double *params, int32_t probe_steps, double dt,
                  double eps_over_ds, int32_t *chosen);
/* Tuned shapes of a context to / from a small text file (path host string). */
int swim_tune_save(swim_ctx *ctx, const char *path);
int swim_tune_load(swim_ctx *ctx, const char *path);

/* One evaluation of the dense velocity sum of eq. (BrV), Sec. 2.1:
 *   u_i = sum_j [ H1(r_ij) F_j + H2(r_ij) (F_j . x_ij) x_ij ],
 * x_ij = X_i - X_j, over all points j of the system of i (self term
 * included), for n_sys independent systems.
 * sys_off  host int64[n_sys+1]: system s owns points [sys_off[s], sys_off[s+1]),
 *          sys_off[0] = 0, non-decreasing.
 * alpha    host double[n_sys], >= 0;  eps host double[n_sys], > 0;
 *          alpha*eps <= 1 (Brinkman length longer than the blob).
 * x,y,fx,fy device dtype[sys_off[n_sys]]: positions and point forces (SoA).
 * ux,uy    device dtype[sys_off[n_sys]]: velocities (written).
 * Errors: SWIM_EINVAL for a bad layout or parameter.  Asynchronous. */
int swim_pair_velocity(swim_ctx *ctx, int32_t dtype, int64_t n_sys, const int64_t *sys_off,
                       const double *alpha, const double *eps, const void *x, const void *y,
                       const void *fx, const void *fy, void *ux, void *uy, void *stream);

/* swim_pair_velocity for callers that cannot allocate memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results, with the call's
 * workspace (system offsets, alpha, eps, block list, per-system constants
 * and FP32 kernel tables) in a fixed device array of the library instead of
 * context allocations, and its few host values copied from the stack by one
 * synchronous copy on the stream (no pinned staging).  It calls no
 * hipMalloc, hipFree or other allocating routine.
 * Limits: n_sys <= 64 systems and at most 4160 pair-kernel blocks (256
 * targets each: about 1M points in all); beyond either, SWIM_EINVAL with a
 * message and nothing launched.  Each GPU holds one copy of the array
 * (about 1.7 MB, kept until the process ends; its address is taken by
 * swim_create for the context's device, else SWIM_ESTATE).  Every call on
 * a GPU uses that GPU's one array: calls that overlap on one GPU (several
 * streams or contexts, host threads) race and must be serialized by the
 * caller.  Returns when the host values are on the device; the kernels run
 * asynchronously on the stream. */
int swim_pair_velocity_noalloc(swim_ctx *ctx, int32_t dtype, int64_t n_sys, const int64_t *sys_off,
                               const double *alpha, const double *eps, const void *x, const void *y,
                               const void *fx, const void *fy, void *ux, void *uy, void *stream);

/* Velocity (eq. BrV) and pressure (eq. BrP) of the n regularized point
 * forces of one system at nt arbitrary target points, for flow and pressure
 * pictures (Sec. 2.1).
 *   u(x) = sum_j [ H1(r) F_j + H2(r) (F_j . d) d ],  d = x - X_j
 *   p(x) = sum_j F_j . grad G_eps(d),  grad G_eps(d) = d m(r) / (2 pi r^2)
 * G_eps solves Delta G_eps = phi, the blob of the velocity kernel, and m(r)
 * is the blob mass inside r: m = r^2/R^2 for alpha = 0 and
 * m = 1 - eps K1(alpha R) / (R K1(alpha eps)) otherwise, R^2 = r^2 + eps^2
 * (with SWIM_BLOB_PAPER: m = 1 - eps^3/R^3 for every alpha).
 * x, y, fx, fy device dtype[n]; tx, ty device dtype[nt]; u, v, p device
 * dtype[nt] (written).  alpha >= 0, eps > 0, alpha*eps <= 1.  Sums are
 * accumulated in FP64.  FP32 reads the pair kernel from the system's table
 * (as the forward runs do; built on the device at each call, for the
 * paper's blob at alpha > 0 from its quadrature), with the direct FP32
 * evaluation beyond it; FP64 evaluates it directly (the paper's blob at
 * alpha > 0: quadrature per pair).  The pressure weight m/(2 pi r^2):
 * FP32 from a second per-call table on the same intervals, FP64 directly.
 * Sums are FP64 either way.  Asynchronous. */
int swim_flow_field(swim_ctx *ctx, int32_t dtype, int64_t n, const void *x, const void *y, const void *fx,
                    const void *fy, double alpha, double eps, int64_t nt, const void *tx, const void *ty,
                    void *u, void *v, void *p, void *stream);

/* Elastic point forces F = -dE/dX (eqs. Fenergy, EFB, curva, EFT) at time t
 * for n_fil filaments stored back to back.
 * N        host int32[n_fil], 3 <= N[f] <= 4096 points of filament f.
 * params   host double[n_fil][SWIM_NPARAM] (alpha, x0, y0 unused here).
 * x,y      device dtype[sum N]; fx,fy device dtype[sum N] (written).
 * Asynchronous. */
int swim_elastic_forces(swim_ctx *ctx, int32_t dtype, int64_t n_fil, const int32_t *N,
                        const double *params, double t, const void *x, const void *y, void *fx,
                        void *fy, void *stream);

/* Forward model g(theta|M) of eq. (model_err): runs n_sys independent
 * systems for `steps` forward-Euler steps of size dt.  System s holds
 * n_swim[s] filaments of N[s] points each (all of one fluid: alpha is taken
 * from its first filament's row).  Each step, at t = step*dt: preferred
 * curvature, forces of every filament, velocity sum over all points of the
 * system, Euler update; after the update, if (step+1) % obs_every == 0, the
 * head X_{N-1} of every filament is stored.
 * N        host int32[n_sys], 3 <= N <= 4096;  n_swim host int32[n_sys] >= 1
 *          or NULL (one filament each); N[s]*n_swim[s] <= 4096.
 * params   device double[n_filaments][SWIM_NPARAM], filaments in system order.
 * eps_over_ds > 0: blob width in units of ds (eps = eps_over_ds / (N-1)).
 * obs      device dtype[n_filaments][steps/obs_every][2] head positions
 *          (NaN for samples a stopped run did not reach); may be NULL if
 *          obs_every == 0.
 * speed    device dtype[n_filaments]: |X_h(T) - X_h(0)| / T, T = steps*dt
 *          (NaN for stopped runs).
 * status   device int32[n_sys]: SWIM_ST_* per system.
 * steps_done device int32[n_sys] or NULL: forward-Euler steps computed per
 *          system (steps, or the step at which the run stopped, 0 if not run).
 * Systems of up to 512 points run in the persistent kernel (a workgroup per
 * system, work queue in longest-first order), one launch per size bucket
 * (systems of up to 64*tpl points, tpl in {1,2,3,4,6,8}); larger systems
 * run the large-system step, launches per Euler step with the work split
 * over workgroups (SWIM_OPT_BIG_TPL).  The buckets and the large systems
 * run side by side on the context's stream and up to three more; with more
 * than four such parts, adjacent buckets closest in size merge (the smaller
 * systems run in the larger bucket's launch) until four remain.  Waves of
 * larger buckets issue at a higher priority where launches share a CU.  FP32 systems whose pairs could lie beyond
 * the FP32 kernel table within the position bound (2829 (N-1) / eps_over_ds
 * >= 2^22, i.e. eps_over_ds well below 1.5) take the large-system step at
 * any size, since the persistent kernel does not test for such pairs.
 * Asynchronous. */
int swim_forward(swim_ctx *ctx, int32_t dtype, int64_t n_sys, const int32_t *N,
                 const int32_t *n_swim, const double *params, int32_t steps, double dt,
                 int32_t obs_every, double eps_over_ds, void *obs, void *speed, int32_t *status,
                 int32_t *steps_done, void *stream);

/* ABC distance: d_i = sqrt(mean over n_obs samples and both coordinates of
 * (obs_i - data)^2); d_i = +inf if status[i] != 0 or d_i is not finite.
 * obs device dtype[n][n_obs][2]; data device double[n_obs][2];
 * status device int32[n] or NULL; dist device double[n] (written).
 * Asynchronous. */
int abc_distance(swim_ctx *ctx, int32_t dtype, int64_t n, int32_t n_obs, const void *obs,
                 const double *data, const int32_t *status, double *dist, void *stream);

/* Percentile tolerance over the completed runs: tol = k-th smallest finite
 * value of dist[0..n), k = ceil(q * n_f) clamped to [1, n_f], n_f the
 * number of finite distances (failed runs carry +inf and are rejected);
 * tol = +inf when n_f = 0.  accept[i] = dist[i] finite and <= tol (ties
 * accepted).
 * dist device double[n]; tol device double[1] (written);
 * accept device uint8[n] (written) or NULL.  Asynchronous. */
int abc_select(swim_ctx *ctx, int64_t n, const double *dist, double q, double *tol,
               uint8_t *accept, void *stream);

/* Prior draw (host, FP64): theta_i[d] = lo[d] + (hi[d]-lo[d]) u, with the
 * uniforms of Philox4x32-10 (Salmon et al. 2011) at key = seed, counter =
 * (i lo, i hi, draw, stream 0), draws 0 and 1.  theta host double[n][dim],
 * dim <= 4. */
int abc_prior_draw(uint64_t seed, int64_t n, int32_t dim, const double *lo, const double *hi,
                   double *theta);

/* PMC proposals for generation `generation` >= 1 (host, FP64): resample the
 * previous population by its weights and perturb with a Gaussian of
 * covariance 2x its weighted covariance (Beaumont et al. 2009); proposals
 * outside [lo, hi] are redrawn (Philox stream 1+generation, attempt a uses
 * draws 3a..3a+2).  prev_theta host double[n_prev][3], prev_w host
 * double[n_prev] (normalized or not); theta host double[n][3]. */
int abc_pmc_propose(uint64_t seed, int32_t generation, int64_t n, const double *prev_theta,
                    const double *prev_w, int64_t n_prev, const double *lo, const double *hi,
                    double *theta);

/* PMC weights (host, FP64): for the accepted proposals (accept[i] != 0),
 * w_i proportional to 1 / sum_j prev_w_j N(theta_i; prev_theta_j, 2 Sigma),
 * Sigma the weighted covariance of the previous population (uniform prior);
 * normalized over the accepted ones; w_i = 0 for rejected ones.
 * theta host double[n][3], accept host uint8[n], w host double[n]. */
int abc_pmc_weights(int64_t n, const double *theta, const uint8_t *accept,
                    const double *prev_theta, const double *prev_w, int64_t n_prev, double *w);

/* One ABC generation end to end (synchronous; host arrays in and out):
 * proposals (prior draw for generation 0, PMC proposals otherwise; host,
 * FP64), forward runs (device, model->dtype), distances, percentile
 * tolerance and acceptance (device), weights (host: 1/n_accepted for
 * generation 0, Beaumont weights otherwise).  The forward runs follow the
 * context's SWIM_OPT_GRAPH mode (a repeated layout, e.g. the generations of
 * one PMC run, is captured once and replayed); use_graph = 0 in the model
 * forces eager launches for this call.
 *   data       host double[n_obs][2], n_obs = model->steps / obs_every;
 *   N          host int32[n], points of particle i;
 *   prev_theta, prev_w  host double[n_prev][3], double[n_prev] (the previous
 *              generation's accepted population; NULL for generation 0);
 *   q          tolerance quantile in (0, 1] over the completed runs;
 *   theta_out  host double[n][3]; dist_out host double[n] (+inf: failed);
 *   accept_out host uint8[n]; w_out host double[n] (0 where rejected);
 *   tol_out    host double[1]; steps_out host int32[n] or NULL (steps each
 *              run completed).
 * SWIM_EINVAL on bad arguments (before any launch). */
typedef struct {
    double lo[3], hi[3];   /* uniform prior box on (alpha, S_b, S_s) */
    double b, omega, k;    /* beat amplitude, angular frequency, wavenumber */
    int32_t steps, obs_every;
    double dt, eps_over_ds;
    int32_t dtype;
    int32_t use_graph;     /* 0: eager launches for this call; 1: the context's graph mode */
} abc_model;

int abc_step(swim_ctx *ctx, const abc_model *model, const double *data, int32_t n_obs, int64_t n,
             const int32_t *N, uint64_t seed, int32_t generation, const double *prev_theta,
             const double *prev_w, int64_t n_prev, double q, double *theta_out, double *dist_out,
             uint8_t *accept_out, double *w_out, double *tol_out, int32_t *steps_out);

/* ---------------------------------------------------------------------------
 * TMCMC (Sec. 2.3, Algorithm TMCMC): transitional Markov chain Monte Carlo
 * over the batched forward model, the sampler the paper uses.
 * ------------------------------------------------------------------------- */

/* Gaussian log-likelihood of forward runs, eqs. (likelihood)-(fitness) with
 * Sigma = sigma_i^2 I over the m = 2 n_obs head coordinates of run i (obs:
 * [n][n_obs][2] in the run's dtype, data: FP64 [n_obs][2], sigma: FP64 [n],
 * status: int32 [n], logl: FP64 [n]; all device pointers):
 * logl_i = -m/2 log(2 pi) - m log(sigma_i) - |D - g_i|^2 / (2 sigma_i^2),
 * -inf where status_i != 0.  Asynchronous on `stream` (NULL: the context's
 * stream).  SWIM_EINVAL for null pointers with n > 0 or n_obs < 1. */
int tmcmc_loglik(swim_ctx *ctx, int32_t dtype, int64_t n, int32_t n_obs, const void *obs, const double *data,
                 const double *sigma, const int32_t *status, double *logl, void *stream);

typedef struct {
    double lo[4], hi[4];   /* uniform prior box on (alpha, S_b, S_s, sigma); sigma: noise std, lo[3] > 0 */
    double cv_target;      /* coefficient of variation of the plausibility weights per stage (1.0) */
    double cov_scale;      /* b: proposal covariance = b^2 x weighted sample covariance (0.2) */
    int32_t max_stages;    /* bound on the number of stages */
} tmcmc_opts;

/* One full TMCMC run (synchronous).  n samples per stage; the forward model
 * of every sample is one swimmer of N points configured by `model` (its
 * b, omega, k, steps, obs_every, dt, eps_over_ds, dtype, use_graph; the
 * prior box comes from `opts`); data: host FP64 [n_obs][2] observed head
 * positions, n_obs = steps / obs_every.
 *
 * Stage j computes the plausibility weights p(D|theta)^dq of the current
 * samples, dq the largest increment (up to 1 - q_j) whose weights have a
 * coefficient of variation of at most cv_target (bisection), S_j = their
 * mean, the normalized weights and b^2 times their weighted covariance.  It
 * then draws n samples by the weights (multinomial), and runs one Metropolis
 * chain per drawn sample, as long as the number of times it was drawn, with
 * target p(D|theta)^q_{j+1} pi(theta) and Gaussian proposals of that
 * covariance.  Proposals outside the box are rejected without a run; runs
 * that stop (blow-up) have zero likelihood.  All chains step together: one
 * batched forward launch per Metropolis step.  The run ends after the
 * stage at q = 1, or after max_stages stages.
 *
 * Outputs (host): theta_out [n][4] and logl_out [n], the final samples and
 * their log-likelihoods; q_out [max_stages + 1] (q_0 = 0, ...,
 * q_{n_stages}); *n_stages_out; *log_evidence_out = sum_j log S_j;
 * accepted_out [max_stages] accepted moves per stage; *runs_out forward runs
 * (may be NULL); *seconds_out wall time of the forward and likelihood calls
 * (may be NULL).  Random numbers: Philox with key seed (prior: stream 0 as
 * abc_prior_draw; resampling of stage j: stream 1000 + 2j; chains of stage
 * j: stream 1001 + 2j).  SWIM_EINVAL for bad arguments or when no prior
 * sample has a finite likelihood. */
int tmcmc_run(swim_ctx *ctx, const abc_model *model, const tmcmc_opts *opts, const double *data, int32_t n_obs,
              int32_t N, int64_t n, uint64_t seed, double *theta_out, double *logl_out, double *q_out,
              int32_t *n_stages_out, double *log_evidence_out, int64_t *accepted_out, int64_t *runs_out,
              double *seconds_out);

/* ---------------------------------------------------------------------------
 * Full sperm model (Appendix, Table Tab:param): a flagellum of n_flag points
 * with the tapered beat, a circular head of n_head points and the neck, with
 * n_swim swimmers in one fluid per system.
 *
 * Geometry of one swimmer, left to right: flagellum point k at (x0 + k ds,
 * y0), ds = 1/(n_flag-1).  The head centre is the last flagellum point
 * shifted right by head_radius + neck_gap.  Head point m sits at angle
 * m 2pi/n_head about that centre, so point n_head/2 (angle pi) is the one
 * nearest the flagellum.
 *
 * Discrete energy (trapezoid rule, centred differences; every spring is
 * K (l/L0 - 1)^2 L0, the trapezoid form of eq. EFT):
 *   flagellum tension  K_T   between neighbours, rest ds
 *   flagellum bending  K_C   sum_{k=1}^{n_flag-2} (zeta_k - zhat_k)^2 ds
 *                      (eqs. EFB, curva), with zhat = d^2/ds^2 of
 *                      a (1-s) sin(eta s - omega t + phase)
 *   head ring          K_HT  neighbouring head points, rest 2 H_r sin(pi/n_head)
 *   head diameters     K_HT  points pi apart, rest 2 H_r
 *   head bending       K_HC  (kappa_m - 1/H_r)^2 times the chord, every node
 *   neck springs       K_NT  last flagellum point to the head points at
 *                      pi - dth, pi, pi + dth; the point before it to
 *                      pi -+ dth; rest = initial lengths
 *   neck angle         K_NA  (z1 . z2)^2, z1 = H(pi) - F(last),
 *                      z2 = H(pi + dth) - H(pi - dth)
 * Forces are F = -dE/dX (eq. Fenergy).  Velocities come from the eq. (BrV)
 * sum over all points of the system, and positions advance by forward
 * Euler (Sec. 2.1).
 * ------------------------------------------------------------------------- */
#define SWIM_SP_ALPHA 0 /* Brinkman resistance alpha >= 0                   */
#define SWIM_SP_KC 1    /* K_C, flagellum curvature stiffness              */
#define SWIM_SP_KT 2    /* K_tens, flagellum tensile stiffness             */
#define SWIM_SP_KHT 3   /* K_H,tens, head tensile stiffness                */
#define SWIM_SP_KHC 4   /* K_H,C, head curvature stiffness                 */
#define SWIM_SP_KNT 5   /* K_N,tens, neck tensile stiffness                */
#define SWIM_SP_KNA 6   /* K_N,ang, neck angle stiffness                   */
#define SWIM_SP_A 7     /* beat amplitude a                                */
#define SWIM_SP_ETA 8   /* beat wavenumber eta                             */
#define SWIM_SP_OMEGA 9 /* beat angular frequency omega                    */
#define SWIM_SP_NPARAM 10

typedef struct swim_sperm_shape {
    int32_t n_flag;     /* points on the flagellum, >= 4                       */
    int32_t n_head;     /* points on the head, even, >= 4                      */
    int32_t n_swim;     /* swimmers per system, >= 1;
                           n_swim * (n_flag + n_head) <= 512                   */
    int32_t reserved;   /* 0                                                   */
    double eps;         /* blob width, > 0                                     */
    double head_radius; /* H_r > 0                                             */
    double neck_gap;    /* dN > 0: gap between the last flagellum point and
                           the head                                            */
} swim_sperm_shape;

/* Runs n_sys independent systems of the full sperm model for `steps`
 * forward-Euler steps of size dt.  Each step, at t = step*dt: forces of
 * every swimmer, velocity sum over all points of the system, Euler update.
 * sys_params  device double[n_sys][SWIM_SP_NPARAM].
 * swim_params device double[n_sys * n_swim][3]: x0, y0 (first flagellum
 *             point) and beat phase of each swimmer, systems in order.
 * head, tail  device dtype[n_sys * n_swim][n_obs + 1][2], n_obs =
 *             steps/obs_every (0 if obs_every == 0).  Sample 0 is the
 *             initial state; sample j follows step j*obs_every.  head is
 *             the head centre (mean of the head points) and tail is the
 *             tail end (flagellum point 0).  Samples a stopped run does not
 *             reach are NaN.
 * status      device int32[n_sys]: SWIM_ST_* per system.  A row with
 *             non-finite values, alpha < 0 or alpha*eps > 1 gets
 *             SWIM_ST_BADPARAM and is not run.
 * Systems run in a persistent kernel, one workgroup per system.
 * SWIM_OPT_WPS set to 2, 4 or 8 selects its waves per system.  Otherwise
 * SWIM_F64 takes 8, and SWIM_F32 the most of 8, 4, 2 that keeps the launch
 * within eight waves per compute unit (small batches are latency-bound).
 * SWIM_EINVAL for a bad shape or run length.  Asynchronous. */
int swim_sperm_forward(swim_ctx *ctx, int32_t dtype, int64_t n_sys, const swim_sperm_shape *shape,
                       const double *sys_params, const double *swim_params, int32_t steps, double dt,
                       int32_t obs_every, void *head, void *tail, int32_t *status, void *stream);

/* Observables of the paper's experiments (Sec. 4) from a swim_sperm_forward
 * run, for samples k = 1..n_obs:
 *   SWIM_OBS_HEAD_VELOCITY   head-centre velocity of swimmer 0,
 *                            (h_k - h_{k-1}) / dt_obs, x then y (Sec. 4.1);
 *   SWIM_OBS_PAIR_DISTANCES  distance between the tail ends, then between
 *                            the head centres, of swimmers 0 and 1 (Secs.
 *                            4.2, 4.3; n_swim >= 2).
 * head, tail device dtype[n_sys * n_swim][n_obs + 1][2] (swim_sperm_forward);
 * status device int32[n_sys]; g device double[n_sys][n_obs][2] (written;
 * NaN for systems whose status is not 0).  Asynchronous. */
#define SWIM_OBS_HEAD_VELOCITY 0
#define SWIM_OBS_PAIR_DISTANCES 1
int swim_sperm_observables(swim_ctx *ctx, int32_t dtype, int32_t kind, int64_t n_sys, int32_t n_swim,
                           int32_t n_obs, double dt_obs, const void *head, const void *tail,
                           const int32_t *status, double *g, void *stream);

/* Gaussian log-likelihood of eqs. (likelihood)-(fitness) with the diagonal
 * covariance of Sec. 4.3.  Entries 0, 2, 4, ... (odd in the paper's 1-based
 * numbering) have standard deviation sigma2[i][0]; entries 1, 3, ... have
 * sigma2[i][1].  Equal values give Sigma = sigma^2 I.
 *   log p = -n_obs log(2 pi) - n_obs (log s_a + log s_b)
 *           - sum_a r^2 / (2 s_a^2) - sum_b r^2 / (2 s_b^2)
 * g device double[n][n_obs][2]; data device double[n_obs][2];
 * sigma2 device double[n][2]; status device int32[n] or NULL.
 * logl device double[n] (written): -inf where status != 0, an output is not
 * finite, or a sigma is not > 0.  Asynchronous. */
int tmcmc_loglik2(swim_ctx *ctx, int64_t n, int32_t n_obs, const double *g, const double *data,
                  const double *sigma2, const int32_t *status, double *logl, void *stream);

/* TMCMC over the full sperm model (Sec. 4).  Each sample's forward run is
 * one system of model->shape.n_swim swimmers placed by swim_rows.
 * theta has n_theta = n_fields + n_sigma entries:
 *   - entries 0 .. n_fields-1 set the system-row fields field[0..]; the
 *     other fields keep sys_row;
 *   - the last n_sigma entries are relative noise levels gamma = sigma/beta
 *     (Sec. 4).  With n_sigma == 1: s_a = gamma beta[0], s_b = gamma beta[1].
 *     With n_sigma == 2: s_a = gamma_a beta[0], s_b = gamma_b beta[1].
 * The likelihood is that of tmcmc_loglik2 on the observables of `kind`.
 * The stages, weights, resampling and chains are those of tmcmc_run over
 * the n_theta parameters. */
typedef struct sperm_tmcmc_model {
    swim_sperm_shape shape;
    double sys_row[SWIM_SP_NPARAM]; /* values of the fields not sampled          */
    int32_t n_theta;                /* 2..4                                      */
    int32_t n_sigma;                /* 1 or 2                                    */
    int32_t field[3];               /* SWIM_SP_* set by theta[0..n_theta-n_sigma) */
    int32_t kind;                   /* SWIM_OBS_*                                */
    double beta[2];                 /* noise scales of entry types a and b, > 0 */
    int32_t steps, obs_every;       /* n_obs = steps / obs_every >= 1            */
    double dt;
    int32_t dtype;                  /* SWIM_F32 or SWIM_F64                      */
    int32_t reserved;               /* 0                                         */
} sperm_tmcmc_model;

/* One full TMCMC run over the sperm model (synchronous).  swim_rows: host
 * double[n_swim][3] (x0, y0, phase) shared by all samples.  data: host
 * double[n_obs][2] observables.  The prior box is opts->lo/hi[0..n_theta);
 * the boxes of the noise levels must have lo >= 0.  Outputs as in tmcmc_run
 * with n_theta columns: theta_out host double[n][n_theta], logl_out
 * double[n], q_out double[max_stages + 1], accepted_out
 * int64[max_stages]; runs_out and seconds_out may be NULL. */
int tmcmc_sperm_run(swim_ctx *ctx, const sperm_tmcmc_model *model, const double *swim_rows,
                    const tmcmc_opts *opts, const double *data, int32_t n_obs, int64_t n, uint64_t seed,
                    double *theta_out, double *logl_out, double *q_out, int32_t *n_stages_out,
                    double *log_evidence_out, int64_t *accepted_out, int64_t *runs_out, double *seconds_out);

/* ---------------------------------------------------------------------------
 * Surrogate of the forward model (not in the paper; prescreens ABC
 * proposals): an MLP 5 -> 256 -> 256 -> 256 -> 256 -> 33 with GELU
 * x Phi(x) on the hidden layers.  Inputs (alpha, ln S_b, ln S_s, b, omega),
 * outputs the head displacement at n_sum observation times (x, y) and the
 * mean speed, all standardized.  BF16 MFMA with FP32 accumulation: every
 * GEMM operand is rounded to bfloat16 (nearest-even); FP32 master weights.
 * Parameters: one FP32 vector of SWIM_MLP_NPARAM values, for each layer
 * l = 0..4 the weights W_l (fan_in x fan_out, row-major) then the bias b_l.
 * --------------------------------------------------------------------------- */
#define SWIM_MLP_NPARAM 207393
#define SWIM_MLP_IN 5
#define SWIM_MLP_OUT 33

/* Y = f(X): X device float[n][5], Y device float[n][33].  Asynchronous. */
int surrogate_forward(swim_ctx *ctx, int64_t n, const float *X, const float *params, float *Y,
                      void *stream);

/* Gradient of the loss mean((f(X) - T)^2) over the n x 33 outputs:
 * grads device float[SWIM_MLP_NPARAM] (parameter layout), loss device float[1]
 * (sum of squares; divide by 33 n) or NULL.  n <= 2^20.  Asynchronous. */
int surrogate_grad(swim_ctx *ctx, int64_t n, const float *X, const float *T, const float *params,
                   float *grads, float *loss, void *stream);

/* Adam training (beta = 0.9, 0.999, eps = 1e-8): epochs x floor(n/batch)
 * steps; step s of epoch e uses the rows perm[e*n + s*batch ...] (device
 * int32[epochs][n], a permutation per epoch supplied by the caller).
 * Row indices outside [0, n) give NaN rows (and a NaN loss), never reads
 * out of bounds.  params, adam_m, adam_v device float[SWIM_MLP_NPARAM],
 * updated in place
 * (m, v start at zero for a fresh run).  loss_out device float[epochs *
 * floor(n/batch)] (per-step sum of squares) or NULL.  Asynchronous. */
int surrogate_train(swim_ctx *ctx, int64_t n, const float *X, const float *T, const int32_t *perm,
                    int32_t epochs, int32_t batch, float lr, float *params, float *adam_m,
                    float *adam_v, float *loss_out, void *stream);

/* Prescreen: d_i = sqrt(mean_j (mu_j + sd_j f(X_i)_j - obs_j)^2) over the
 * first n_sum outputs; keep[i] = d_i <= tol; idx[0..*n_keep) = the kept i in
 * ascending order.  X device float[n][5]; out_mu, out_sd, obs_sum device
 * float (de-standardization and observed summaries); dist device float[n]
 * or NULL; keep device uint8[n]; idx device int64[n]; n_keep device
 * int64[1].  Asynchronous. */
int surrogate_prescreen(swim_ctx *ctx, int64_t n, const float *X, const float *params,
                        const float *out_mu, const float *out_sd, const float *obs_sum,
                        int32_t n_sum, float tol, float *dist, uint8_t *keep, int64_t *idx,
                        int64_t *n_keep, void *stream);

/* X[i] = (alpha, ln S_b, ln S_s, b, omega) of theta device double[n][3],
 * standardized with mu, sd (device float[5]) unless both are NULL. */
int surrogate_features(swim_ctx *ctx, int64_t n, const double *theta, double b, double omega,
                       const float *mu, const float *sd, float *X, void *stream);

/* T[i] = (obs_i[idx_j] - (x0, y0) for j < n_sum, speed_i): device
 * float[n][2 n_sum + 1] from a forward run's obs / speed (dtype). */
int surrogate_targets(swim_ctx *ctx, int32_t dtype, int64_t n, int32_t n_obs, const void *obs,
                      const void *speed, double x0, double y0, const int32_t *sum_idx,
                      int32_t n_sum, float *T, void *stream);

/* Column mean and population standard deviation (1 if zero) of A device
 * float[n][cols] into mu, sd device float[cols]; standardize in place. */
int surrogate_colstats(swim_ctx *ctx, int64_t n, int32_t cols, const float *A, float *mu,
                       float *sd, void *stream);
int surrogate_standardize(swim_ctx *ctx, int64_t n, int32_t cols, float *A, const float *mu,
                          const float *sd, void *stream);

/* abc_prior_draw on the device: theta device double[n][3], identical values. */
int abc_prior_draw_device(swim_ctx *ctx, uint64_t seed, int64_t n, const double *lo,
                          const double *hi, double *theta, void *stream);

/* Parameter rows (alpha, S_b, S_s, b, omega, k, 0, 0, 0) for swim_forward
 * from theta rows idx[j] (idx NULL: row j), j < min(cap, *n_dev) (n_dev
 * NULL: cap), theta device double[n_theta][3].  An index outside
 * [0, n_theta) gives a NaN row, which swim_forward flags
 * SWIM_ST_BADPARAM.  All device.  Asynchronous. */
int swim_param_rows(swim_ctx *ctx, int64_t cap, const int64_t *n_dev, const int64_t *idx,
                    int64_t n_theta, const double *theta, double b, double omega, double k,
                    double *rows, void *stream);

/* keep[i] = values[i] == want (values NULL: keep given), then idx[0..*n_keep)
 * = the kept i in ascending order.  All device.  Asynchronous. */
int swim_select(swim_ctx *ctx, int64_t n, const int32_t *values, int32_t want, uint8_t *keep,
                int64_t *idx, int64_t *n_keep, void *stream);

/* dst[j] = src[idx[j]] (rows of cols floats), j < min(cap, *n_dev); src
 * device float[n_src][cols]; an index outside [0, n_src) gives a NaN row.
 * Device.  Asynchronous. */
int swim_gather_rows(swim_ctx *ctx, int64_t cap, const int64_t *n_dev, const int64_t *idx,
                     int64_t n_src, const float *src, int32_t cols, float *dst, void *stream);

/* Training set of the surrogate, end to end on the device: n_runs prior
 * draws (abc_prior_draw values, Philox seed), one forward run each with N
 * points (model's steps, dt, dtype), inputs (alpha, ln S_b, ln S_s, b,
 * omega) and targets (head displacement from its start (1, 0) at the
 * observation indices sum_idx[0..n_sum), then the mean speed).  Runs that
 * did not complete (status != 0), or whose head moved farther than
 * max_disp (> 0) from its start in either coordinate at a summary time (an
 * Euler instability still below the blow-up bound), are dropped; the first
 * min(kept, cap) kept runs, in draw order, are written to X (device float[cap][5])
 * and T (device float[cap][33]) standardized by their own column mean and
 * standard deviation, returned in in_mu, in_sd (device float[5]) and
 * out_mu, out_sd (device float[33]).  n_sum must be 16; *n_out (host) =
 * rows written.  Synchronizes once (for the count). */
int surrogate_dataset(swim_ctx *ctx, const abc_model *model, int32_t N, int64_t n_runs,
                      uint64_t seed, const int32_t *sum_idx, int32_t n_sum, double max_disp,
                      int64_t cap, float *X, float *T, float *in_mu, float *in_sd, float *out_mu,
                      float *out_sd, int64_t *n_out, void *stream);

/* Surrogate-prescreened rejection ABC, end to end (synchronous; runs on the
 * context's stream).  n_prop prior draws (abc_prior_draw values, Philox
 * seed) on the device; the surrogate (params, input and output
 * standardization) predicts their summaries, and those whose surrogate
 * distance to the observed summaries (data at sum_idx minus the head's
 * start (1, 0)) is <= factor * tol survive.  The first min(survivors, cap)
 * survivors, in draw order, are re-run on the plain forward model (N
 * points, model's steps, dt, dtype) and accepted when their ABC distance to
 * data (host double[n_obs][2]) is finite and <= tol.  The tolerance being
 * known, a re-run stops (status SWIM_ST_REJECTED, distance +inf) once the
 * running sum of its squared head deviations from the data exceeds
 * 2 n_obs tol^2 (1 + 1e-6): that sum only grows, so the run's distance
 * would exceed tol (SWIM_OPT_EARLY_STOP = 0 runs every survivor to the
 * end; the accepted set is the same).  Host outputs:
 * theta_out double[cap][3], dist_out double[cap], accept_out uint8[cap],
 * *n_surv = survivors (may exceed cap), ms_out float[2] (prescreen and
 * re-run milliseconds on the device) or NULL. */
int abc_prescreened(swim_ctx *ctx, const abc_model *model, int32_t N, const float *params,
                    const float *in_mu, const float *in_sd, const float *out_mu,
                    const float *out_sd, const int32_t *sum_idx, int32_t n_sum, const double *data,
                    int32_t n_obs, double tol, double factor, int64_t n_prop, uint64_t seed,
                    int64_t cap, double *theta_out, double *dist_out, uint8_t *accept_out,
                    int64_t *n_surv, float *ms_out);

/* Host evaluation of the device kernel functions (test hook): for squared
 * distances t[0..n) returns H1(t) - H1(0) and H2(t) as computed by the
 * kernels' own code compiled for the host, and H1(0) in *h1c.  SWIM_F32
 * follows the FP32 device path: cubic pieces of a per-system table in
 * v = 1 + sigma t (sigma the power of four with sigma eps^2 in [1, 4);
 * 16 pieces per octave, v < 2^44), built from the FP64 evaluation; direct
 * FP32 evaluation beyond.  blob: SWIM_BLOB_READING or SWIM_BLOB_PAPER (as
 * SWIM_OPT_BLOB); SWIM_EINVAL otherwise. */
int swim_kernel_eval_host(int32_t dtype, double alpha, double eps, int32_t blob, int64_t n, const double *t,
                          double *h1t, double *h2, double *h1c);

/* Launch plan of a swim_forward call (host only, no device work): for each
 * system, the targets per lane of the persistent-kernel launch it runs in
 * (1, 2, 3, 4, 6 or 8, after the merging of size buckets that swim_forward
 * describes), or -1 for the large-system step.  Arguments as swim_forward's
 * (N, n_swim host; n_swim may be NULL); tpl host int32[n_sys] (written).
 * SWIM_EINVAL for a bad dtype or sizes outside swim_forward's limits. */
int swim_forward_plan(int32_t dtype, int64_t n_sys, const int32_t *N, const int32_t *n_swim,
                      double eps_over_ds, int32_t *tpl);

#ifdef __cplusplus
}
#endif

#endif /* SWIM_H */
