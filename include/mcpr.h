/*
 * mcpr.h -- C ABI of the MI355X fine propagator and MC-moments Parareal driver
 * (Bossuyt, Vandewalle, Samaey, "Monte-Carlo/Moments micro-macro Parareal
 * method for unimodal and bimodal scalar McKean-Vlasov SDEs", arXiv 2310.11365).
 *
 * Conventions shared by every call
 *   - Device pointers (particle arrays, statistics, maps) are owned by the
 *     caller; the library never frees them.  Host pointers are read or written
 *     only for the duration of the call.
 *   - Calls taking a stream are asynchronous on that stream (a hipStream_t;
 *     NULL is the null stream) unless stated otherwise.  Kernels of one call
 *     run in stream order; a context must not be used from two host threads or
 *     two streams at once (it owns the reduction scratch).
 *   - Particle arrays hold n_particles values of type double (MCPR_FP64) or
 *     float (MCPR_FP32) and must be 16-byte aligned.
 *   - Every call validates its arguments before launching anything and
 *     returns MCPR_E_INVALID_ARG (nothing launched) on a bad argument;
 *     mcpr_last_error() then describes it.  HIP failures give MCPR_E_DEVICE.
 *   - Random numbers: Philox4x32-10 with key = (seed low word, seed high
 *     word) and counter = (p / 4, step or boundary index, instance, tag);
 *     particle p takes word p % 4, Box-Muller pairs words (0,1) and (2,3).
 *     Tags: 0 Euler-Maruyama, 1 initial normal, 2 initial mixture pick,
 *     3 matching resample.  The numbers depend on the particle, the global step
 *     and the instance only, so every Parareal iteration and the serial run see
 *     the same numbers (Property "Exactness of MC-moments Parareal").
 */
#ifndef MCPR_H
#define MCPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mcpr_ctx mcpr_ctx;
typedef struct mcpr_parareal mcpr_parareal;
typedef void *mcpr_stream; /* hipStream_t */

typedef enum {
    MCPR_OK = 0,
    MCPR_E_INVALID_ARG = -1,
    MCPR_E_OOM = -2,
    MCPR_E_DEVICE = -3,
    MCPR_E_NONFINITE = -4,
    MCPR_E_UNSUPPORTED = -5,
    MCPR_E_NOT_RESERVED = -6 /* the context's scratch is smaller than the call needs: see mcpr_reserve */
} mcpr_status;

enum { MCPR_FP64 = 0, MCPR_FP32 = 1 }; /* FP32: fp32 particles, fp64 reductions and matching */
enum { MCPR_P0_NORMAL = 0, MCPR_P0_MIXTURE = 1, MCPR_P0_DELTA = 2 };
enum { MCPR_MAP_KEEP = 0, MCPR_MAP_AFFINE = 1, MCPR_MAP_RESAMPLE = 2 };
enum { MCPR_MAX_REGIONS = 8 };
/* Coarse moment models: the Taylor model (eq. moment_model_class_1) or the
 * Gaussian assumed-density model (eq. Gaussian_model_McK_V_SDE) with its
 * expectations by Gauss-Hermite sigma points, 2 (exact to degree 3) or 3
 * (exact to degree 5, i.e. exact Gaussian closure for the supported cubic
 * drift and affine diffusion).                                              */
enum { MCPR_COARSE_TAYLOR = 0, MCPR_COARSE_GAUSS2 = 1, MCPR_COARSE_GAUSS3 = 2 };

/* Drift and diffusion of the scalar McKean-Vlasov SDE (Sec. 1.1, eq.
 * general_McKean_Vlasov) in the class this library supports: polynomial in
 * the particle position, affine in the ensemble's mean m and variance v, plus
 * the terms below (x E[X^2], trigonometric, empirical CDF).
 *   a(x, m, v) = a0 + a1 x + a2 x^2 + a3 x^3 + am m + av v
 *   b(x, m, v) = b0 + b1 x + bm m + bv v                                    */
typedef struct {
    double a0, a1, a2, a3, am, av;
    double b0, b1, bm, bv;
    double axs; /* drift term axs * x * E[X^2], E[X^2] = v + m^2 (the polynomial-drift
                   example of App. on the exactness of the moment model); the
                   adjoint needs axs = 0 */
    /* Trigonometric drift terms ksin sin x + kc E_q[sin(X_q - x)], where the
     * mean-field average is (1/P) sum_q sin(X_q - x) = S cos x - C sin x with
     * S, C the population means of sin X and cos X (the plane rotator of
     * Sec. 5.1: ksin = -1, kc = K).  With either nonzero the per-step mean
     * field is (S, C) instead of (m, v), so am, av, axs, bm and bv must be 0
     * (else MCPR_E_UNSUPPORTED), and the adjoint refuses the problem.        */
    double ksin, kc;
    /* Empirical-CDF drift term acdf (1 - F_P(x)), F_P(x) = (1/P) sum_q H(x - X_q)
     * with the step function H(0) = 1/2 (the Burgers example of Sec. 5.2:
     * acdf = 1, b0 = sigma, X(0) = 0).  With acdf nonzero every step sorts
     * each ensemble (mcpr_set_cdf_sort; at most 2^32 - 2 particles in one
     * call, else MCPR_E_UNSUPPORTED), the problem has one region, the
     * Taylor (Gaussian-density) coarse model and no wrap, and the other
     * mean-field coefficients (am, av, axs, bm, bv, ksin, kc) must be 0, else
     * MCPR_E_UNSUPPORTED; the adjoint refuses the problem.                    */
    double acdf;
} mcpr_coef;

/* One problem: coefficients, initial law p0, time grid, regions of
 * attraction (Sec. 2.2: D_i = [split_{i-1}, split_i), split_0 = -inf,
 * split_I = +inf; a particle on a boundary belongs to the upper region).    */
typedef struct {
    mcpr_coef coef;
    int32_t p0_kind;   /* MCPR_P0_*: N(mu1, sd1^2); w N(mu1,sd1^2) + (1-w) N(mu2,sd2^2); point mass at mu1 */
    int32_t precision; /* MCPR_FP64 or MCPR_FP32 */
    double p0_w, p0_mu1, p0_sd1, p0_mu2, p0_sd2;
    double dt;               /* Euler-Maruyama step; a slice is steps_per_slice steps */
    int32_t steps_per_slice; /* m >= 1 */
    int32_t n_slices;        /* N >= 1 */
    int32_t n_regions;       /* I, 1..MCPR_MAX_REGIONS */
    int32_t coarse_substeps; /* RK4 steps per slice of the coarse propagator, >= 1 */
    double split[MCPR_MAX_REGIONS - 1]; /* I-1 increasing boundaries */
    uint64_t seed;
    int32_t coarse_model;    /* MCPR_COARSE_*: moment model of the coarse propagator */
    int32_t wrap;            /* 1: after every Euler-Maruyama step each particle is shifted modulo
                                2 pi into [0, 2 pi) (the plane rotator's convention); 0: none */
} mcpr_problem;

/* One particle ensemble (a micro state u in R^P, Sec. 3.4). */
typedef struct {
    void *x;             /* device, n_particles values, 16-byte aligned          */
    int64_t n_particles; /* P >= 1                                              */
    int32_t instance;    /* RNG stream (counter word 2), >= 0                    */
    int32_t slice;       /* slice index n: step j draws at global step n*m + j   */
    int32_t problem;     /* index into the problems[] array of the call          */
    int32_t reserved;
} mcpr_ensemble;

/* Restriction record of one region (eq. multimodal_R): particle count,
 * population mean and variance (weights 1/n), min and max.  n == 0: mean,
 * var are 0.  If all particles of the region coincide, var is exactly 0 and
 * mean is that value.  nonfinite != 0 if any particle was NaN or Inf.      */
typedef struct {
    int64_t n;
    double mean, var, min, max;
    int32_t nonfinite;
    int32_t reserved;
} mcpr_region_stats;

/* Matching of the particles of one region (eq. multimodal_M):
 *   MCPR_MAP_KEEP      x' = x
 *   MCPR_MAP_AFFINE    x' = fma(scale, x - from, to)     (sqrt(sigma/V[u]) (u - E[u]) + mu)
 *   MCPR_MAP_RESAMPLE  x' = fma(scale, xi, to)           (sqrt(sigma) xi + mu, V[u] = 0)
 * xi: tag-3 normals at counter word 1 = boundary.  In MCPR_FP32 the map is
 * evaluated in fp64 and rounded once to fp32.                              */
typedef struct {
    double from, scale, to;
    int32_t mode;
    int32_t boundary;
} mcpr_region_map;

/* ---- context ------------------------------------------------------------ */
/* Creates a context on a HIP device; it owns the scratch of the calls
 * (reduction partials, work tables, pinned staging of the tables, the
 * adjoint's checkpoints), sized by mcpr_reserve: the calls below never
 * allocate, synchronise the device or free memory for scratch; a call that
 * needs more than is reserved returns MCPR_E_NOT_RESERVED and launches
 * nothing.  (Events of the profiling hooks and of the launch-variant trial,
 * and the graph of a new launch shape, are created on first use.)          */
mcpr_status mcpr_create(mcpr_ctx **ctx, int32_t device);
void mcpr_destroy(mcpr_ctx *ctx);
const char *mcpr_last_error(const mcpr_ctx *ctx); /* NULL: the calling thread's last context-free call */
const char *mcpr_version(void);

/* Sizes the context's scratch for later calls of the kinds in `calls` on the
 * given ensembles, or on any set that needs no more (fewer or smaller
 * ensembles of the same layout): allocates device and pinned host memory and
 * may synchronise the device, so call it outside the hot path.  Buffers only
 * grow; a reserve that fits what is held allocates nothing.  Kinds:
 *   MCPR_RESERVE_INIT     mcpr_init_particles
 *   MCPR_RESERVE_MOMENTS  mcpr_moments
 *   MCPR_RESERVE_QOI      mcpr_qoi
 *   MCPR_RESERVE_FINE     mcpr_fine_propagate, with records and trace
 *   MCPR_RESERVE_MATCH    mcpr_match, with the dry-run probe
 *   MCPR_RESERVE_ADJOINT  mcpr_adjoint from each given ensemble (its slice to
 *                         n_slices), with the backward sweep
 * mcpr_parareal_create reserves everything its driver needs itself.  Errors:
 * as the calls (arguments), MCPR_E_OOM when an allocation fails.           */
enum {
    MCPR_RESERVE_INIT = 1,
    MCPR_RESERVE_MOMENTS = 2,
    MCPR_RESERVE_QOI = 4,
    MCPR_RESERVE_FINE = 8,
    MCPR_RESERVE_MATCH = 16,
    MCPR_RESERVE_ADJOINT = 32,
    MCPR_RESERVE_ALL = 63
};
mcpr_status mcpr_reserve(mcpr_ctx *ctx, const mcpr_problem *problems, int32_t n_problems, const mcpr_ensemble *ens,
                         int32_t n_ens, int32_t calls);
/* Allocations the context (and its Parareal drivers) has made so far: device
 * and pinned host buffers, and their bytes (either pointer may be NULL).    */
mcpr_status mcpr_alloc_stats(const mcpr_ctx *ctx, int64_t *allocations, int64_t *bytes);

/* Quantity of interest (Sec. 1.1: the sample average of Phi over the
 * ensemble; Sec. 5.1 uses Phi(x) = sin(x^2) for the geometric Brownian motion
 * example): out[e] = (1/P) sum_p Phi(x_p) of ensemble e, Phi evaluated in
 * fp64 from the state, summed in the canonical order.  out: device array
 * [n_ens].  Asynchronous.  Errors: MCPR_E_INVALID_ARG for an unknown kind or
 * a null out, and as mcpr_fine_propagate for the ensembles.                  */
enum { MCPR_QOI_X = 0, MCPR_QOI_X2 = 1, MCPR_QOI_SIN_X2 = 2 };
mcpr_status mcpr_qoi(mcpr_ctx *ctx, const mcpr_problem *problems, int32_t n_problems, const mcpr_ensemble *ens,
                     int32_t n_ens, int32_t kind, double *out, mcpr_stream stream);

/* Measurement: when enabled, each fine sweep brackets its run of
 * Euler-Maruyama step launches with a pair of HIP events on the call's
 * stream (launched directly, not from a graph).  mcpr_profile_read waits for
 * the recorded events and returns the summed elapsed time of those runs,
 * the number of step launches and the particle-steps done.                  */
mcpr_status mcpr_profile_enable(mcpr_ctx *ctx, int32_t on);
mcpr_status mcpr_profile_read(mcpr_ctx *ctx, double *em_ms, int64_t *em_launches, int64_t *particle_steps,
                              int32_t reset);
/* The same for mcpr_adjoint's backward sweep: one event pair around each
 * slice's run of backward step launches; returns their summed time, the
 * number of backward steps and the particle-steps they covered.             */
mcpr_status mcpr_profile_read_adjoint(mcpr_ctx *ctx, double *ms, int64_t *launches, int64_t *particle_steps,
                                      int32_t reset);

/* Measurement: the HBM streaming ceiling of the step kernel's access pattern
 * (the bound its roofline fraction is read against besides the vendor
 * peak).  reps in-place passes x <- 1.0f * x over n floats (device, 16-byte
 * aligned, n a multiple of 4096; contents unchanged) with the step kernel's
 * block shape (256 threads x 4 quads, non-temporal loads and stores), after
 * one warm-up pass; ms_per_pass (host) receives the mean time of a pass,
 * i.e. 8 n bytes moved.  Takes no context; synchronises the stream; errors
 * as the context-free calls (mcpr_last_error(NULL)).                        */
mcpr_status mcpr_stream_probe(void *x, int64_t n, int32_t reps, mcpr_stream stream, double *ms_per_pass);

/* hipGraph replay of the fine sweep (on by default): the launch sequence of/* hipGraph replay of the fine sweep (on by default): the launch sequence of
 * a fine sweep (step-0 sums, the steps, the final moments and records) is
 * captured once per shape into a graph on a library-owned stream and
 * replayed; the caller's stream waits on it through events.  Results are
 * bitwise the same as direct launches.  A sweep with the empirical-CDF drift
 * (acdf != 0) is always launched directly: it calls the library sort.
 * mcpr_graph_stats: graphs built and replays so far.                        */
mcpr_status mcpr_set_graphs(mcpr_ctx *ctx, int32_t on);

/* Step-kernel launch variants, all giving the same bits: bit 0 non-temporal
 * loads and stores of the state (pays off when the state does not fit the
 * Infinity Cache), bit 1 the step's mean field formed once per ensemble by a
 * small launch instead of by every block (pays off with many blocks per
 * ensemble).  mode -1 (default): the first fine sweep of each launch shape
 * (with at least 8 steps) runs each candidate variant on consecutive steps of
 * its first 16 (8 if it has fewer than 16), times each by its launches after
 * the first (which inherits the previous candidate's cache state), and adopts
 * a candidate other than the first for that shape only if it beats the first
 * by 1 %.  Candidates: 0..3, or only 2 and 3 when an ensemble of the launch
 * has more than 256 superchunks (more than 1048576 particles), where 2 is
 * also the untuned default.  0..3 forces a variant.  The trigonometric and
 * empirical-CDF steps have one kernel each: no variants, no trial.
 * mcpr_tuned_variant: the variant chosen for the index-th tuned shape, or -1. */
mcpr_status mcpr_set_tuning(mcpr_ctx *ctx, int32_t mode);
int32_t mcpr_tuned_variant(const mcpr_ctx *ctx, int32_t index);
mcpr_status mcpr_graph_stats(const mcpr_ctx *ctx, int64_t *builds, int64_t *launches);

/* Resident fine sweeps (eq. Euler_Maruyama with the per-step mean field of
 * Sec. 2, the same arithmetic and the same bits as the per-step launches).
 * When every ensemble of an mcpr_fine_propagate call (or of a Parareal
 * iteration's sweep) has at most 12288 particles and neither the
 * trigonometric nor the empirical-CDF term, the sweep runs in two launches:
 * the normals of all its steps (into library scratch of at most 256 MB,
 * sized by mcpr_reserve; a call whose normals do not fit what was reserved
 * runs the per-step launches instead), then one block per ensemble that
 * keeps the particles in registers through all the steps and reduces each
 * step's mean field inside the block in the canonical order.  A step then
 * costs one block barrier instead of a launch (the latency-bound regime of
 * small ensembles).
 * mcpr_set_resident: 1 (default) allows it, 0 always uses per-step launches.
 * mcpr_resident_sweeps: fine sweeps run resident so far.                    */
mcpr_status mcpr_set_resident(mcpr_ctx *ctx, int32_t enable);
mcpr_status mcpr_resident_sweeps(const mcpr_ctx *ctx, int64_t *sweeps);

/* Sort of the empirical-CDF drift (acdf != 0; Sec. 5.2: every step needs
 * each ensemble in ascending order).  mode 1 (default): the first two steps
 * of a fine sweep sort with a device-wide radix sort, later steps put the new
 * states into buckets between the previous step's sorted states (1792 apart
 * on average) and sort each bucket on chip (a bitonic network in one
 * wavefront's registers for a bucket of up to 2048 states, in one block for a
 * larger one).  A bucket beyond 4096 states (a
 * law still spreading fast, as in the first steps from a point mass; a point
 * mass without noise) makes the sweep run again with the radix sort on its
 * first 8 steps, then 32, then all of them; the overflow flag is read after
 * the first bucket step and at the end of the sweep.  A call with this drift
 * synchronises its stream (to read the flag).
 * mode 0: the device-wide radix sort on every step.  Both give the same bits.
 * mcpr_cdf_stats: sweeps done by the buckets, by the radix sort alone, and
 * sweeps redone after an overflow, so far (any pointer may be NULL).        */
mcpr_status mcpr_set_cdf_sort(mcpr_ctx *ctx, int32_t mode);
mcpr_status mcpr_cdf_stats(const mcpr_ctx *ctx, int64_t *bucket_sweeps, int64_t *library_sweeps,
                           int64_t *redone_sweeps);

/* ---- hot-path calls ------------------------------------------------------ */
/* Initial law p0 (Sec. 1.1) sampled into each ensemble (tags 1 and 2). */
mcpr_status mcpr_init_particles(mcpr_ctx *ctx, const mcpr_problem *problems, int32_t n_problems,
                                const mcpr_ensemble *ens, int32_t n_ens, mcpr_stream stream);

/* Restriction R (eq. multimodal_R; S of Sec. 3.4 when I = 1).
 * stats: device, [n_ens][n_regions + 1]; entry n_regions is the whole ensemble.
 * Ensembles of one call must share n_regions. */
mcpr_status mcpr_moments(mcpr_ctx *ctx, const mcpr_problem *problems, int32_t n_problems,
                         const mcpr_ensemble *ens, int32_t n_ens, mcpr_region_stats *stats,
                         mcpr_stream stream);

/* Fine propagator F_n (eq. Euler_Maruyama, with the X_n term of the standard
 * scheme): steps_per_slice Euler-Maruyama steps of every ensemble, in place,
 * all ensembles batched into each step's launch.  Step j of ensemble e uses
 * the population mean and variance of e at the start of the step (the
 * empirical measure of eq. general_equation) and normals at global step
 * slice*m + j.  Ensembles of one call must share steps_per_slice, precision
 * and n_regions; their coefficients and sizes may differ.
 * stats (device, may be NULL): [n_ens][n_regions + 1] restriction of the
 *   final state.
 * trace (device, may be NULL): [n_ens][steps_per_slice + 1][2]: entry j <
 *   m is the (mean, variance) step j used, entry m the mean and variance of
 *   the final state.                                                       */
mcpr_status mcpr_fine_propagate(mcpr_ctx *ctx, const mcpr_problem *problems, int32_t n_problems,
                                const mcpr_ensemble *ens, int32_t n_ens, mcpr_region_stats *stats,
                                double *trace, mcpr_stream stream);

/* The fine propagator of mcpr_fine_propagate for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels, launch order and
 * results bit for bit (the untuned default launch variant, no graph replay),
 * with every scratch buffer in a static device array of the library
 * (4 MiB per device, held until the process ends; its address is looked up
 * once per device on the first call there) instead of a context.  Takes no
 * context; the work tables are written by kernels from their arguments, so
 * nothing is copied from host memory.  stats and trace (may be NULL) are
 * written directly, same layout as mcpr_fine_propagate.  Asynchronous on
 * stream, on the calling thread's current device.
 * Limits: the scratch must hold 256-byte-aligned parts of n_ens work items
 * (264 B each), and per superchunk (4096 particles, or 1024 below 65536
 * particles) 40 B plus, with stats, 40 B per region and one more: about
 * 1.4e8 particles in one call with stats and one region, 1e8 with two.  A
 * call needing more returns MCPR_E_INVALID_ARG and launches nothing; the
 * empirical-CDF drift
 * (acdf != 0) returns MCPR_E_UNSUPPORTED.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (two host threads, two streams) race and give wrong results.
 * Errors: as mcpr_fine_propagate; the text is mcpr_last_error(NULL), per host
 * thread.                                                                    */
mcpr_status mcpr_fine_propagate_static(const mcpr_problem *problems, int32_t n_problems, const mcpr_ensemble *ens,
                                       int32_t n_ens, mcpr_region_stats *stats, double *trace, mcpr_stream stream);

/* Matching T per region (eq. multimodal_M), in place.  maps: device,
 * [n_ens][n_regions].  dry_run != 0: nothing is written; probe (device,
 * [n_ens][n_regions + 1]) receives the restriction of the transformed values
 * grouped by the region each particle came from (min and max decide whether
 * a region stays inside its domain, Remark on particle fractions).         */
mcpr_status mcpr_match(mcpr_ctx *ctx, const mcpr_problem *problems, int32_t n_problems,
                       const mcpr_ensemble *ens, int32_t n_ens, const mcpr_region_map *maps,
                       int32_t dry_run, mcpr_region_stats *probe, mcpr_stream stream);

/* Pathwise gradient of the slice-end moments through the fine propagator
 * (discrete adjoint of the Euler-Maruyama scheme with the noise fixed; not in
 * the paper, used to fit coarse-model and fraction-model parameters).
 * Runs the serial fine solution of slices ens->slice .. n_slices-1 from the
 * state ens->x (not modified), with a checkpoint at every slice start, and
 * reports the (mean, variance) at each slice end (host moments_out
 * [n][2], may be NULL).  If dL_dmoments (host [n][2], upstream derivatives
 * of a scalar L with respect to those moments) is given, the backward sweep
 * recomputes each slice once from its checkpoint (on the context's second
 * stream, overlapped with the backward steps of the following slice) and
 * writes grad_out (host [10]) = dL/d(a0, a1, a2, a3, am, av, b0, b1, bm, bv).
 * With graphs on (mcpr_set_graphs) and profiling off, the whole launch
 * sequence is captured once per shape and replayed; every per-call value
 * (work tables, moments, dL_dmoments) is read from device memory, so the
 * results are those of direct launches.  fp64 adjoint state and reductions;
 * synchronises the stream.  Scratch (sized by mcpr_reserve with
 * MCPR_RESERVE_ADJOINT): (n + 1) + 2 (m + 1) states, two fp64 arrays of P,
 * the per-slice work tables.                                                 */
mcpr_status mcpr_adjoint(mcpr_ctx *ctx, const mcpr_problem *problem, const mcpr_ensemble *ens,
                         const double *dL_dmoments, double *moments_out, double *grad_out, mcpr_stream stream);

/* ---- Parareal driver ----------------------------------------------------- */
/* One Parareal instance: an independent problem with its own particle count
 * and ring of n_slices + 1 ensemble slots (caller-owned device memory of
 * (n_slices + 1) * slot_stride values; slot_stride >= n_particles and a
 * multiple of 4).  Slice n of iteration k lives in slot (n - k) mod (N + 1).*/
typedef struct {
    int32_t problem;  /* index into problems[] */
    int32_t instance; /* RNG stream */
    int64_t n_particles;
    int64_t slot_stride;
    void *ring;
} mcpr_instance;

/* Generalised micro-macro Parareal (eq. mM_parareal_other_k_NEW) with the
 * MC-moments iterator (unimodal and multimodal definitions of Sec. 3.4;
 * alpha = (a - c) + R(b)), lifting by T of u0, coarse propagator = Taylor
 * moment model (eq. moment_model_class_1 per region, eq.
 * moment_model_Taylor_multimodal) with fractions frozen, RK4.  learning != 0:
 * the particle-fraction model of Sec. 3.6 (two regions).  All instances of
 * one driver share steps_per_slice, n_slices, n_regions and precision.  The
 * problems array is copied.  An instance stops iterating once its delta
 * (below) is <= tol, or after n_slices iterations (every slice exact).      */
mcpr_status mcpr_parareal_create(mcpr_ctx *ctx, const mcpr_problem *problems, int32_t n_problems,
                                 const mcpr_instance *inst, int32_t n_inst, int32_t learning, double tol,
                                 mcpr_parareal **out);
void mcpr_parareal_destroy(mcpr_parareal *pr);

/* Iteration 0: if sample_u0, draw u0 from p0 into slot 0 (else slot 0 must
 * hold u0); rho_0 = R(u0); rho^0_{n+1} = C_n(rho^0_n); u^0_n = T(rho^0_n, u0)
 * per region.  Waits for the records of u0 (the host needs them) and returns
 * with the lifting queued on the stream. */
mcpr_status mcpr_parareal_init(mcpr_parareal *pr, int32_t sample_u0, mcpr_stream stream);

/* One iteration k -> k+1 for every instance that has not stopped: F on the
 * slices n >= k of all instances in one batched sweep, sequential coarse
 * sweep with the iterator on the host, matching on the device.  delta_out
 * (host, may be NULL): [n_inst] max over n of the change of the global mean
 * and variance.  Waits for the sweep's records (the host needs them) and
 * returns with the matching queued on the stream: synchronise the stream
 * before reading the ring. */
mcpr_status mcpr_parareal_iterate(mcpr_parareal *pr, double *delta_out, mcpr_stream stream);

/* Number of iterations done (k). */
int32_t mcpr_parareal_iteration(const mcpr_parareal *pr);

/* Quantity of interest of every slice of the current iterate of instance
 * inst: out (host) [N+1], out[n] = (1/P) sum Phi over u^k_n (mcpr_qoi).  The
 * ring holds slices k..N only; the slices below k are exact and their values
 * come from the QoI recorded when each became exact, which needs tracking
 * (mcpr_parareal_track_qoi) switched on before mcpr_parareal_init, else
 * MCPR_E_INVALID_ARG once k > 0.  Synchronises the stream. */
mcpr_status mcpr_parareal_qoi(mcpr_parareal *pr, int32_t inst, int32_t kind, double *out, mcpr_stream stream);

/* QoI tracking: when on, init and every iterate also queue the QoI (every
 * kind) of the slice that has just become exact (three small reductions of
 * one ensemble per instance). */
mcpr_status mcpr_parareal_track_qoi(mcpr_parareal *pr, int32_t on);

/* Given particle fractions for instance inst (the reference variant of
 * Sec. 5.3 that uses the exact particle fractions, e.g. those of a serial
 * fine solution, in place of the Parareal approximations): fractions is a
 * host array [(N+1)][I], copied.  From the next mcpr_parareal_init or
 * mcpr_parareal_iterate on, every macro state rho^k_n carries fractions[n]
 * (after the learning override, if any); the cached coarse outputs keep the
 * fractions they were computed with, so exact slices still take the I(a,b,a)
 * branch.  NULL returns to the method's own fractions.  Errors:
 * MCPR_E_INVALID_ARG for a bad instance or a negative or non-finite value. */
mcpr_status mcpr_parareal_set_fractions(mcpr_parareal *pr, int32_t inst, const double *fractions);

/* Checkpoint and resume between iterations.  The driver's state is its host
 * state (this call) plus the instances' rings, which are caller-owned device
 * memory: a caller saves the rings (slots of slices k..N of each instance,
 * or simply the whole ring) with the state and copies them back before
 * mcpr_parareal_restore.  Random numbers are counter-based, so iterations
 * after a restore give the same bits as an uninterrupted run.
 * mcpr_parareal_save: *bytes receives the state's size; with buf != NULL and
 * capacity >= that size the state is written to buf (host).  Call between
 * iterations; it waits for the QoI still in flight.
 * mcpr_parareal_restore: loads a state saved from a driver created with the
 * same problems, instances (particle counts, RNG streams), N, m, regions and
 * precision, in this process or another; anything else returns
 * MCPR_E_INVALID_ARG and leaves the driver as it was.                       */
mcpr_status mcpr_parareal_save(mcpr_parareal *pr, void *buf, size_t capacity, size_t *bytes);
mcpr_status mcpr_parareal_restore(mcpr_parareal *pr, const void *buf, size_t bytes);

/* Macro state of instance i (host arrays): rho [(N+1)][I][3] = (fraction,
 * mean, variance) per region; glob [(N+1)][2] = mixture mean and variance
 * (eq. mixture_of_distributions_mean_variance).  Either may be NULL. */
mcpr_status mcpr_parareal_macro(const mcpr_parareal *pr, int32_t inst, double *rho, double *glob);

/* Iterator outcome of the last iteration, [N][I] (host): 0 short cut
 * I(a,b,a) = (R(b), b), 1 matched, 2 negative variance, 3 would leave its
 * region, 4 empty region. */
mcpr_status mcpr_parareal_flags(const mcpr_parareal *pr, int32_t inst, int32_t *flags);

/* Device pointer of u^k_n (slice-start state n of the current iteration k of
 * instance inst, which stops counting when it reaches its tolerance).  Only
 * slices n >= k are held (the ring has N+1 slots); n < k gives
 * MCPR_E_INVALID_ARG. */
mcpr_status mcpr_parareal_slot(const mcpr_parareal *pr, int32_t inst, int32_t n, void **x);

#ifdef __cplusplus
}
#endif

#endif /* MCPR_H */
