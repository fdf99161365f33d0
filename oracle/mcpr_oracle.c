/*
 * mcpr_oracle.c -- plain FP64 CPU oracle for the Monte-Carlo/moments
 * micro-macro Parareal method of Bossuyt, Vandewalle and Samaey (arXiv
 * 2310.11365) on scalar McKean-Vlasov SDEs.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it is used by tests/, by __graft_entry__.smoke() and by the
 * cpu_baseline leg of bench.py, and by nothing else.  It shares no source with
 * the HIP library (its own Philox, its own structs, its own driver).
 *
 * Style: scalar loops, double precision everywhere, long double accumulators
 * for sums, two-pass moments, no blocking or fusion.  Build with
 *   gcc -O2 -ffp-contract=off -fPIC -shared
 * so that every a*b+c is two rounded operations, exactly as written.
 *
 * What each function computes, and the passage it follows:
 *   or_philox4x32_10   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The
 *                      paper names no generator; it only needs the same
 *                      numbers in every iteration (Property "Exactness of
 *                      MC-moments Parareal", Sec. 5 protocol).
 *   or_normals4        Box-Muller on the four words of one Philox call.
 *   or_sample_p0       initial law p0 of the SDE (Sec. 1.1, Sec. 5.3 setups).
 *   or_qoi             empirical mean of a quantity of interest Phi (Sec. 1.1;
 *                      Phi(x) = sin(x^2) in the geometric Brownian motion
 *                      example of Sec. 5.2).
 *   or_restrict        restriction R: per-region fraction, mean, variance
 *                      (eq. multimodal_R) and the mixture moments
 *                      (eq. mixture_of_distributions_mean_variance).
 *   or_fine            fine propagator F_n: Euler-Maruyama (eq. Euler_Maruyama)
 *                      on the P-particle system (eq. general_equation).
 *   or_coarse          coarse propagator C_n: Taylor moment model
 *                      (eq. moment_model_class_1, derivation App. D) or the
 *                      Gaussian model with sigma points (eq.
 *                      Gaussian_model_McK_V_SDE), one pair per region
 *                      (eq. moment_model_Taylor_multimodal), RK4.
 *   or_transform       matching T (eq. multimodal_M).
 *   or_parareal        generalised micro-macro Parareal
 *                      (eq. mM_parareal_other_k_NEW) with the unimodal and
 *                      multimodal MC-moments iterators (Definitions of Sec. 3.4),
 *                      the learning extension (Sec. 3.6) and the reference
 *                      variant with given (exact) particle fractions (the
 *                      variants listed in Sec. 5.3).
 *   or_fraction_fit    least-squares fit of the two-region rate model
 *                      (eq. exponential_for_particle_fractions, App. H).
 *   or_adjoint         pathwise gradient of a moment-misfit through the
 *                      Euler-Maruyama scheme (not in the paper; the gradient
 *                      of the discrete scheme, derived by hand).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Problem description (the oracle's own; mirrors the paper's ingredients:    */
/* drift a, diffusion b, p0, slices, time step, regions of attraction).       */
/* ------------------------------------------------------------------------- */
typedef struct {
    /* drift a(x, m, v) = a0 + a1 x + a2 x^2 + a3 x^3 + am m + av v          */
    double a0, a1, a2, a3, am, av;
    /* diffusion b(x, m, v) = b0 + b1 x + bm m + bv v                         */
    double b0, b1, bm, bv;
    /* drift term axs x E[X^2] with E[X^2] = v + m^2 (polynomial drift of the
       appendix on the exactness of the moment model)                        */
    double axs;
    /* trigonometric drift ksin sin x + kc (1/P) sum_q sin(X_q - x), the
       second written as kc (S cos x - C sin x) with S, C the population means
       of sin X and cos X (plane rotator of Sec. 5.1)                         */
    double ksin, kc;
    /* empirical-CDF drift acdf (1 - F_P(x)), F_P(x) = (1/P) sum_q H(x - X_q),
       H(0) = 1/2 (Burgers example of Sec. 5.2)                              */
    double acdf;
    /* initial law: kind 0 = N(mu1, sd1^2), 1 = w N(mu1,sd1^2) + (1-w) N(mu2,sd2^2),
       2 = point mass at mu1                                                  */
    int32_t p0_kind, pad0;
    double p0_w, p0_mu1, p0_sd1, p0_mu2, p0_sd2;
    double dt;                 /* Euler-Maruyama step                          */
    int32_t steps_per_slice;   /* m: slice length Delta T = m * dt             */
    int32_t n_slices;          /* N                                            */
    int32_t n_regions;         /* I, 1..8                                      */
    int32_t coarse_substeps;   /* RK4 steps per slice                          */
    double split[7];           /* region boundaries, increasing                */
    uint64_t seed;
    int32_t coarse_model;      /* 0 Taylor, 1 Gaussian 2-point, 2 Gaussian 3-point */
    int32_t wrap;              /* 1: shift each particle modulo 2 pi into [0, 2 pi) after every step */
} or_problem;

#define OR_TWO_PI 6.283185307179586 /* the double nearest 2 pi */

/* the trigonometric mean field (S, C) replaces (m, v) as the per-step mean field */
static int or_is_trig(const or_problem *pr) { return pr->ksin != 0.0 || pr->kc != 0.0; }

typedef struct {
    int64_t n;
    double mean, var, min, max;
} or_stats;

/* ------------------------------------------------------------------------- */
/* Philox4x32-10                                                              */
/* ------------------------------------------------------------------------- */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Counter layout: (quad index q = p / 4, step or boundary index s, instance,
   tag).  Key: the 64-bit seed split into its low and high words.           */
enum { OR_TAG_EM = 0, OR_TAG_INIT_NORMAL = 1, OR_TAG_INIT_PICK = 2, OR_TAG_MATCH = 3 };

static void or_words(uint64_t seed, uint32_t q, uint32_t s, uint32_t inst, uint32_t tag, uint32_t w[4])
{
    uint32_t ctr[4] = {q, s, inst, tag};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    or_philox4x32_10(ctr, key, w);
}

/* uniform in (0,1): (w + 1/2) / 2^32, exact in double */
double or_uniform(uint32_t w)
{
    return ((double)w + 0.5) / 4294967296.0;
}

/* Four standard normals from one Philox call: Box-Muller on the pairs
   (u0,u1) and (u2,u3).                                                      */
void or_normals4(uint64_t seed, uint32_t q, uint32_t s, uint32_t inst, uint32_t tag, double z[4])
{
    const double two_pi = 6.283185307179586476925286766559;
    uint32_t w[4];
    or_words(seed, q, s, inst, tag, w);
    double u0 = or_uniform(w[0]), u1 = or_uniform(w[1]);
    double u2 = or_uniform(w[2]), u3 = or_uniform(w[3]);
    double r01 = sqrt(-2.0 * log(u0));
    double r23 = sqrt(-2.0 * log(u2));
    z[0] = r01 * cos(two_pi * u1);
    z[1] = r01 * sin(two_pi * u1);
    z[2] = r23 * cos(two_pi * u3);
    z[3] = r23 * sin(two_pi * u3);
}

static double or_normal_of(uint64_t seed, int64_t p, uint32_t s, uint32_t inst, uint32_t tag)
{
    double z[4];
    or_normals4(seed, (uint32_t)(p >> 2), s, inst, tag, z);
    return z[p & 3];
}

/* ------------------------------------------------------------------------- */
/* Initial law p0                                                             */
/* ------------------------------------------------------------------------- */
void or_sample_p0(const or_problem *pr, int64_t P, uint32_t inst, double *x)
{
    for (int64_t p = 0; p < P; p++) {
        if (pr->p0_kind == 2) {
            x[p] = pr->p0_mu1;
            continue;
        }
        double z = or_normal_of(pr->seed, p, 0u, inst, OR_TAG_INIT_NORMAL);
        if (pr->p0_kind == 0) {
            x[p] = pr->p0_mu1 + pr->p0_sd1 * z;
        } else {
            uint32_t w[4];
            or_words(pr->seed, (uint32_t)(p >> 2), 0u, inst, OR_TAG_INIT_PICK, w);
            double u = or_uniform(w[p & 3]);
            if (u < pr->p0_w)
                x[p] = pr->p0_mu1 + pr->p0_sd1 * z;
            else
                x[p] = pr->p0_mu2 + pr->p0_sd2 * z;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Moments                                                                    */
/* ------------------------------------------------------------------------- */
/* population mean and variance (weights 1/P: the empirical measure of the
   particle system), two passes, extended-precision accumulators             */
void or_moments(const double *x, int64_t P, double *mean, double *var)
{
    long double s = 0.0L;
    for (int64_t p = 0; p < P; p++)
        s += (long double)x[p];
    double m = (double)(s / (long double)P);
    long double s2 = 0.0L;
    for (int64_t p = 0; p < P; p++) {
        long double d = (long double)x[p] - (long double)m;
        s2 += d * d;
    }
    *mean = m;
    *var = (double)(s2 / (long double)P);
}

/* Empirical mean of a quantity of interest over the ensemble, (1/P) sum
   Phi(x_p) (Sec. 1.1, the sample average of Phi; the nonlinear QoI of the
   geometric Brownian motion example of Sec. 5.1 is Phi(x) = sin(x^2)).
   kind 0: x, 1: x^2, 2: sin(x^2).                                            */
double or_qoi(const double *x, int64_t P, int32_t kind)
{
    long double s = 0.0L;
    for (int64_t p = 0; p < P; p++) {
        double v = x[p];
        double phi = kind == 0 ? v : (kind == 1 ? v * v : sin(v * v));
        s += (long double)phi;
    }
    return (double)(s / (long double)P);
}

/* region of x: D_i = [split_{i-1}, split_i), split_0 = -inf, split_I = +inf;
   a particle exactly on a boundary belongs to the upper region               */
int or_region_of(const or_problem *pr, double x)
{
    int r = 0;
    for (int i = 0; i < pr->n_regions - 1; i++)
        if (x >= pr->split[i])
            r = i + 1;
    return r;
}

/* Restriction: per region count, mean, variance, min, max; entry I is the
   whole ensemble.  An empty region has n = 0 and zero mean and variance.  A
   region whose particles all coincide has variance exactly 0 and mean equal
   to that common value (the case "V[u] = 0" of the matching operator).     */
void or_restrict(const or_problem *pr, const double *x, int64_t P, or_stats *out)
{
    int I = pr->n_regions;
    for (int i = 0; i <= I; i++) {
        long double s = 0.0L;
        int64_t n = 0;
        double mn = INFINITY, mx = -INFINITY;
        for (int64_t p = 0; p < P; p++) {
            if (i < I && or_region_of(pr, x[p]) != i)
                continue;
            s += (long double)x[p];
            n++;
            if (x[p] < mn) mn = x[p];
            if (x[p] > mx) mx = x[p];
        }
        or_stats st;
        st.n = n;
        st.min = mn;
        st.max = mx;
        if (n == 0) {
            st.mean = 0.0;
            st.var = 0.0;
        } else if (mn == mx) {
            st.mean = mn;
            st.var = 0.0;
        } else {
            double m = (double)(s / (long double)n);
            long double s2 = 0.0L;
            for (int64_t p = 0; p < P; p++) {
                if (i < I && or_region_of(pr, x[p]) != i)
                    continue;
                long double d = (long double)x[p] - (long double)m;
                s2 += d * d;
            }
            st.mean = m;
            st.var = (double)(s2 / (long double)n);
        }
        out[i] = st;
    }
}

/* ------------------------------------------------------------------------- */
/* Coefficients                                                               */
/* ------------------------------------------------------------------------- */
static double or_drift(const or_problem *pr, double x, double m, double v, double S, double C)
{
    return ((pr->a3 * x + pr->a2) * x + pr->a1) * x + (pr->a0 + pr->am * m + pr->av * v) +
           pr->axs * x * (v + m * m) + pr->ksin * sin(x) + pr->kc * (S * cos(x) - C * sin(x));
}

/* Empirical CDF with the step function H(0) = 1/2 at every particle:
   F[p] = (1/P) sum_q H(x_p - x_q) = (#{q : x_q < x_p} + #{q : x_q = x_p} / 2) / P,
   counted by sorting: the particles of a run of equal values [s, t) in sorted
   order have s smaller ones and t - s equal ones (themselves included).      */
typedef struct {
    double x;
    int64_t i;
} or_keyed;

static int or_cmp_keyed(const void *a, const void *b)
{
    const or_keyed *u = (const or_keyed *)a, *w = (const or_keyed *)b;
    if (u->x < w->x) return -1;
    if (u->x > w->x) return 1;
    return (u->i > w->i) - (u->i < w->i);
}

void or_empirical_cdf(const double *x, int64_t P, double *F)
{
    or_keyed *k = (or_keyed *)malloc(sizeof(or_keyed) * (size_t)P);
    for (int64_t p = 0; p < P; p++) {
        k[p].x = x[p];
        k[p].i = p;
    }
    qsort(k, (size_t)P, sizeof(or_keyed), or_cmp_keyed);
    int64_t s = 0;
    while (s < P) {
        int64_t t = s + 1;
        while (t < P && k[t].x == k[s].x)
            t++;
        double cnt = (double)s + 0.5 * (double)(t - s);
        for (int64_t r = s; r < t; r++)
            F[k[r].i] = cnt / (double)P;
        s = t;
    }
    free(k);
}

static double or_diffusion(const or_problem *pr, double x, double m, double v)
{
    return pr->b1 * x + (pr->b0 + pr->bm * m + pr->bv * v);
}

/* ------------------------------------------------------------------------- */
/* Fine propagator: m Euler-Maruyama steps of slice n, in place.  Step j of  */
/* slice n draws its normals at global step index s = n*m + j, so that every */
/* Parareal iteration and the serial run use the same numbers.  The mean     */
/* field is the population mean and variance at the start of each step.     */
/* With trigonometric drift terms the mean field is (S_j, C_j), the means   */
/* of sin X and cos X, instead.  If trace is non-NULL it receives the mean   */
/* field of each step, j = 0..m-1.  wrap: x <- x - 2 pi floor(x / (2 pi))    */
/* after every step.                                                          */
/* ------------------------------------------------------------------------- */
void or_fine(const or_problem *pr, double *x, int64_t P, uint32_t inst, int32_t slice, double *trace)
{
    int32_t msteps = pr->steps_per_slice;
    double dt = pr->dt;
    double sdt = sqrt(dt);
    int trig = or_is_trig(pr);
    double *F = pr->acdf != 0.0 ? (double *)malloc(sizeof(double) * (size_t)P) : NULL;
    for (int32_t j = 0; j < msteps; j++) {
        uint32_t s = (uint32_t)(slice * msteps + j);
        double mj = 0.0, vj = 0.0, Sj = 0.0, Cj = 0.0;
        if (trig) {
            long double ss = 0.0L, cs = 0.0L;
            for (int64_t p = 0; p < P; p++) {
                ss += (long double)sin(x[p]);
                cs += (long double)cos(x[p]);
            }
            Sj = (double)(ss / (long double)P);
            Cj = (double)(cs / (long double)P);
        } else {
            or_moments(x, P, &mj, &vj);
        }
        if (trace) {
            trace[2 * j] = trig ? Sj : mj;
            trace[2 * j + 1] = trig ? Cj : vj;
        }
        if (F)
            or_empirical_cdf(x, P, F);
        for (int64_t p = 0; p < P; p++) {
            double z = or_normal_of(pr->seed, p, s, inst, OR_TAG_EM);
            double a = or_drift(pr, x[p], mj, vj, Sj, Cj);
            if (F)
                a += pr->acdf * (1.0 - F[p]);
            double b = or_diffusion(pr, x[p], mj, vj);
            x[p] = x[p] + a * dt + b * sdt * z;
            if (pr->wrap)
                x[p] = x[p] - OR_TWO_PI * floor(x[p] / OR_TWO_PI);
        }
    }
    free(F);
}

/* ------------------------------------------------------------------------- */
/* Coarse propagator: for each region the Taylor moment model                */
/*   dM_i/dt = a(M_i, mbar, vbar) + a_xx(M_i) V_i / 2                         */
/*   dV_i/dt = (2 a_x(M_i) + b_x^2) V_i + b(M_i, mbar, vbar)^2                */
/* with the particle fractions frozen over the slice, and (mbar, vbar) the   */
/* mixture mean and variance of the regional moments.  Classical RK4 with    */
/* coarse_substeps equal steps over Delta T = m * dt.                        */
/* y = (M_1, V_1, ..., M_I, V_I); f = fractions.                             */
/* ------------------------------------------------------------------------- */
static void or_mixture(int I, const double *f, const double *y, double *mbar, double *vbar)
{
    double m = 0.0;
    for (int i = 0; i < I; i++)
        if (f[i] > 0.0)
            m += f[i] * y[2 * i];
    double v = 0.0;
    for (int i = 0; i < I; i++)
        if (f[i] > 0.0) {
            double d = y[2 * i] - m;
            v += f[i] * (y[2 * i + 1] + d * d);
        }
    *mbar = m;
    *vbar = v;
}

/* Sigma points of N(M, V) for the Gaussian models (Gauss-Hermite): two
   points M +- sqrt(V), weights 1/2 (exact to degree 3); three points M,
   M +- sqrt(3V), weights 2/3, 1/6, 1/6 (exact to degree 5).  A negative V
   places the points as for V = 0.  Returns the number of points.           */
static int or_sigma_points(int model, double M, double V, double *xs, double *ws)
{
    double Vp = V > 0.0 ? V : 0.0;
    if (model == 1) {
        xs[0] = M - sqrt(Vp); xs[1] = M + sqrt(Vp);
        ws[0] = 0.5; ws[1] = 0.5;
        return 2;
    }
    xs[0] = M - sqrt(3.0 * Vp); xs[1] = M; xs[2] = M + sqrt(3.0 * Vp);
    ws[0] = 1.0 / 6.0; ws[1] = 2.0 / 3.0; ws[2] = 1.0 / 6.0;
    return 3;
}

/* Gaussian assumed-density model (eq. Gaussian_model_McK_V_SDE, with the
   variance integrand read as 2 (x - M) a + b^2): the expectations over
   N(M_i, V_i) by the sigma points.                                         */
static void or_gaussian_rhs(const or_problem *pr, double M, double V, double mbar, double vbar,
                            double S, double C, double *dM, double *dV)
{
    double xs[3], ws[3];
    int K = or_sigma_points(pr->coarse_model, M, V, xs, ws);
    double ea = 0.0, exa = 0.0, eb2 = 0.0;
    for (int k = 0; k < K; k++) {
        double a = or_drift(pr, xs[k], mbar, vbar, S, C);
        double b = or_diffusion(pr, xs[k], mbar, vbar);
        ea += ws[k] * a;
        exa += ws[k] * (xs[k] - M) * a;
        eb2 += ws[k] * b * b;
    }
    *dM = ea;
    *dV = 2.0 * exa + eb2;
}

/* Trigonometric mean field of a macro state: S = sum_i f_i E_i[sin X],
   C = sum_i f_i E_i[cos X], with E_i taken at the region's mean (the Taylor
   model, which gives the paper's plane-rotator moment model) or by the
   region's sigma points (Gaussian models).                                  */
static void or_trig_field(const or_problem *pr, const double *f, const double *y, double *S, double *C)
{
    int I = pr->n_regions;
    double s = 0.0, c = 0.0;
    for (int i = 0; i < I; i++) {
        if (!(f[i] > 0.0))
            continue;
        if (pr->coarse_model == 0) {
            s += f[i] * sin(y[2 * i]);
            c += f[i] * cos(y[2 * i]);
        } else {
            double xs[3], ws[3];
            int K = or_sigma_points(pr->coarse_model, y[2 * i], y[2 * i + 1], xs, ws);
            for (int k = 0; k < K; k++) {
                s += f[i] * ws[k] * sin(xs[k]);
                c += f[i] * ws[k] * cos(xs[k]);
            }
        }
    }
    *S = s;
    *C = c;
}

static void or_coarse_rhs(const or_problem *pr, const double *f, const double *y, double *dy)
{
    int I = pr->n_regions;
    double mbar, vbar, S = 0.0, C = 0.0;
    or_mixture(I, f, y, &mbar, &vbar);
    if (or_is_trig(pr))
        or_trig_field(pr, f, y, &S, &C);
    if (pr->coarse_model == 1 || pr->coarse_model == 2) {
        for (int i = 0; i < I; i++)
            or_gaussian_rhs(pr, y[2 * i], y[2 * i + 1], mbar, vbar, S, C, &dy[2 * i], &dy[2 * i + 1]);
        return;
    }
    for (int i = 0; i < I; i++) {
        double M = y[2 * i], V = y[2 * i + 1];
        double A = or_drift(pr, M, mbar, vbar, S, C);
        double Ax = pr->a1 + 2.0 * pr->a2 * M + 3.0 * pr->a3 * M * M + pr->axs * (vbar + mbar * mbar) +
                    pr->ksin * cos(M) - pr->kc * (S * sin(M) + C * cos(M));
        double Axx = 2.0 * pr->a2 + 6.0 * pr->a3 * M - pr->ksin * sin(M) - pr->kc * (S * cos(M) - C * sin(M));
        double B = or_diffusion(pr, M, mbar, vbar);
        double Bx = pr->b1;
        dy[2 * i] = A + 0.5 * Axx * V;
        dy[2 * i + 1] = (2.0 * Ax + Bx * Bx) * V + B * B;
        if (pr->acdf != 0.0) {
            /* density assumed N(M, V): 1 - CDF(M) = 1/2, d(1 - CDF)/dx at M =
               -1/sqrt(2 pi V), second derivative 0 (the Burgers moment model) */
            double Vp = V > 0.0 ? V : 0.0;
            dy[2 * i] += 0.5 * pr->acdf;
            dy[2 * i + 1] += -2.0 * pr->acdf * sqrt(Vp) / sqrt(2.0 * 3.141592653589793);
        }
    }
}

void or_coarse(const or_problem *pr, const double *f, const double *y_in, double *y_out)
{
    int n = 2 * pr->n_regions;
    double y[16], k1[16], k2[16], k3[16], k4[16], t[16];
    memcpy(y, y_in, sizeof(double) * n);
    double h = (pr->dt * pr->steps_per_slice) / pr->coarse_substeps;
    for (int s = 0; s < pr->coarse_substeps; s++) {
        or_coarse_rhs(pr, f, y, k1);
        for (int i = 0; i < n; i++) t[i] = y[i] + 0.5 * h * k1[i];
        or_coarse_rhs(pr, f, t, k2);
        for (int i = 0; i < n; i++) t[i] = y[i] + 0.5 * h * k2[i];
        or_coarse_rhs(pr, f, t, k3);
        for (int i = 0; i < n; i++) t[i] = y[i] + h * k3[i];
        or_coarse_rhs(pr, f, t, k4);
        for (int i = 0; i < n; i++)
            y[i] = y[i] + (h / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
    memcpy(y_out, y, sizeof(double) * n);
}

/* ------------------------------------------------------------------------- */
/* Matching T([mu, sigma], u) on the particles of one region                 */
/*   sqrt(sigma) xi + mu                              if V[u] = 0            */
/*   sqrt(sigma / V[u]) (u - E[u]) + mu               otherwise              */
/* xi are tag-MATCH normals at the boundary index of the state produced.     */
/* Returns 1 if every transformed particle of the region stays in the        */
/* region, 0 otherwise; writes to y (may equal x) only if apply != 0.        */
/* ------------------------------------------------------------------------- */
int or_transform(const or_problem *pr, const double *x, double *y, int64_t P, uint32_t inst,
                 int32_t boundary, int region, const or_stats *src, double mu, double sigma, int apply)
{
    int inside = 1;
    int degenerate = (src->min == src->max);
    double scale = degenerate ? sqrt(sigma) : sqrt(sigma / src->var);
    for (int64_t p = 0; p < P; p++) {
        if (or_region_of(pr, x[p]) != region)
            continue;
        double xn;
        if (degenerate)
            xn = scale * or_normal_of(pr->seed, p, (uint32_t)boundary, inst, OR_TAG_MATCH) + mu;
        else
            xn = scale * (x[p] - src->mean) + mu;
        if (or_region_of(pr, xn) != region)
            inside = 0;
        if (apply)
            y[p] = xn;
    }
    return inside;
}

/* ------------------------------------------------------------------------- */
/* Macro state helpers: rho = (f_i, M_i, V_i) for i = 0..I-1                  */
/* ------------------------------------------------------------------------- */
static void or_rho_from_stats(int I, int64_t P, const or_stats *st, double *rho)
{
    for (int i = 0; i < I; i++) {
        rho[3 * i] = (double)st[i].n / (double)P;
        rho[3 * i + 1] = st[i].mean;
        rho[3 * i + 2] = st[i].var;
    }
}

/* global mean and variance of a macro state, eq. (mixture of distributions) */
void or_rho_global(int I, const double *rho, double *M, double *V)
{
    double f[8], y[16];
    for (int i = 0; i < I; i++) {
        f[i] = rho[3 * i];
        y[2 * i] = rho[3 * i + 1];
        y[2 * i + 1] = rho[3 * i + 2];
    }
    or_mixture(I, f, y, M, V);
}

/* C_n applied to a macro state: fractions unchanged, regional (M, V) by RK4 */
static void or_coarse_rho(const or_problem *pr, const double *rho, double *out)
{
    int I = pr->n_regions;
    double f[8] = {0}, y[16] = {0}, yo[16] = {0};
    for (int i = 0; i < I; i++) {
        f[i] = rho[3 * i];
        y[2 * i] = rho[3 * i + 1];
        y[2 * i + 1] = rho[3 * i + 2];
    }
    or_coarse(pr, f, y, yo);
    for (int i = 0; i < I; i++) {
        out[3 * i] = f[i];
        out[3 * i + 1] = yo[2 * i];
        out[3 * i + 2] = yo[2 * i + 1];
    }
}

/* ------------------------------------------------------------------------- */
/* Learning: fit P_1(t) = Pstar + (P_1(0) - Pstar) exp(-kappa t) to fraction */
/* data (t_j, y_j) by Levenberg-Marquardt on (kappa, Pstar), P_1(0) = y_0.   */
/* kappa = omega_12 + omega_21, Pstar = omega_21 / kappa: the solution of the */
/* two-region linear rate model dP/dt = A P of App. H.                      */
/* ------------------------------------------------------------------------- */
static double or_frac_model(double y0, double kappa, double pstar, double t)
{
    return pstar + (y0 - pstar) * exp(-kappa * t);
}

static double or_frac_sse(int n, const double *t, const double *y, double kappa, double pstar)
{
    double s = 0.0;
    for (int j = 0; j < n; j++) {
        double r = or_frac_model(y[0], kappa, pstar, t[j]) - y[j];
        s += r * r;
    }
    return s;
}

void or_fraction_fit(int n, const double *t, const double *y, double kappa0, double pstar0,
                     double *kappa_out, double *pstar_out)
{
    double kappa = kappa0, pstar = pstar0, lam = 1e-3;
    double sse = or_frac_sse(n, t, y, kappa, pstar);
    int done = 0;
    for (int it = 0; it < 200 && !done; it++) {
        /* Gauss-Newton normal equations, damped: (J^T J + lam diag(J^T J)) s = -J^T r */
        double g0 = 0, g1 = 0, h00 = 0, h01 = 0, h11 = 0;
        for (int j = 0; j < n; j++) {
            double e = exp(-kappa * t[j]);
            double r = or_frac_model(y[0], kappa, pstar, t[j]) - y[j];
            double dk = -(y[0] - pstar) * t[j] * e;   /* d model / d kappa */
            double dp = 1.0 - e;                       /* d model / d pstar */
            g0 += dk * r;
            g1 += dp * r;
            h00 += dk * dk;
            h01 += dk * dp;
            h11 += dp * dp;
        }
        int improved = 0;
        for (int tries = 0; tries < 40 && !improved; tries++) {
            double a00 = h00 * (1.0 + lam), a11 = h11 * (1.0 + lam), a01 = h01;
            double det = a00 * a11 - a01 * a01;
            if (!(det > 0.0) || !isfinite(det)) {
                lam *= 10.0;
                continue;
            }
            double sk = -(a11 * g0 - a01 * g1) / det;
            double sp = -(a00 * g1 - a01 * g0) / det;
            double kn = kappa + sk, pn = pstar + sp;
            if (kn < 0.0) kn = 0.0;
            if (pn < 0.0) pn = 0.0;
            if (pn > 1.0) pn = 1.0;
            double sn = or_frac_sse(n, t, y, kn, pn);
            if (sn < sse) {
                double step = fabs(kn - kappa) + fabs(pn - pstar);
                double size = fabs(kappa) + fabs(pstar);
                kappa = kn;
                pstar = pn;
                sse = sn;
                lam = (lam / 10.0 > 1e-12) ? lam / 10.0 : 1e-12;
                improved = 1;
                if (step <= 1e-14 * size)
                    done = 1;
            } else {
                lam *= 10.0;
            }
        }
        if (!improved)
            done = 1;
    }
    *kappa_out = kappa;
    *pstar_out = pstar;
}

/* ------------------------------------------------------------------------- */
/* Serial fine solution: u_{n+1} = F_n(u_n), restriction at every boundary.  */
/* x: P particles, u_0 on entry, u_N on exit.  st_out: (N+1) x (I+1).        */
/* ------------------------------------------------------------------------- */
void or_serial(const or_problem *pr, double *x, int64_t P, uint32_t inst, or_stats *st_out)
{
    int I = pr->n_regions;
    or_restrict(pr, x, P, st_out);
    for (int32_t n = 0; n < pr->n_slices; n++) {
        or_fine(pr, x, P, inst, n, NULL);
        or_restrict(pr, x, P, st_out + (size_t)(n + 1) * (I + 1));
    }
}

/* ------------------------------------------------------------------------- */
/* MC-moments Parareal.                                                      */
/*                                                                           */
/* Arrays (all caller-owned):                                                */
/*   u0       P initial particles (unchanged)                                 */
/*   rho_out  (K+1) x (N+1) x I x 3 macro states rho^k_n, k = 0..K           */
/*   glob_out (K+1) x (N+1) x 2 global (mean, variance) of rho^k_n            */
/*   flags    K x N x I iterator outcome for slice n, region i at iteration k */
/*            0: I(a,b,a) short cut, 1: matched, 2: negative variance,       */
/*            3: would leave its region, 4: empty region                     */
/*   delta    K successive-iterate differences (max over n of |dM|, |dV|)    */
/*   states   optional (K+1) x (N+1) x P: u^k_n (n = 0..N; entries of        */
/*            slices already exact are copied from their exact values)       */
/* learning != 0 enables the particle-fraction model (two regions only).     */
/* frac (optional, (N+1) x I): given particle fractions; every macro state   */
/* rho^k_n then carries frac[n] as its fractions (set after rho^k_n is       */
/* formed, after the learning override), while the cached coarse outputs    */
/* keep the fractions they were computed with.  With the fractions of the   */
/* serial fine solution this is the paper's exact-fraction reference.       */
/* Returns the number of iterations performed (stops at K, or when delta <=  */
/* tol, or when every slice is exact).                                       */
/* ------------------------------------------------------------------------- */
int or_parareal(const or_problem *pr, const double *u0, int64_t P, uint32_t inst, int32_t K,
                double tol, int32_t learning, const double *frac, double *rho_out, double *glob_out,
                int32_t *flags, double *delta, double *states)
{
    int N = pr->n_slices, I = pr->n_regions;
    size_t RS = (size_t)I * 3;
    double *cur = (double *)malloc(sizeof(double) * (size_t)(N + 1) * P);   /* u^k_n      */
    double *fine = (double *)malloc(sizeof(double) * (size_t)(N + 1) * P);  /* F(u^k_n)   */
    double *rho = (double *)malloc(sizeof(double) * (N + 1) * RS);          /* rho^k_n    */
    double *nrho = (double *)malloc(sizeof(double) * (N + 1) * RS);
    double *cache = (double *)malloc(sizeof(double) * (N + 1) * RS);        /* C_n(rho^k_n) */
    double *ncache = (double *)malloc(sizeof(double) * (N + 1) * RS);
    or_stats *rec = (or_stats *)malloc(sizeof(or_stats) * (N + 1) * (I + 1)); /* R(F(u^k_n)) */
    double kappa = 0.0, pstar = 0.0;
    int have_fit = 0;

    /* iteration 0: rho^0_0 = R(u0); rho^0_{n+1} = C_n(rho^0_n); u^0_n = L(rho^0_n) */
    or_stats st0[9];
    or_restrict(pr, u0, P, st0);
    or_rho_from_stats(I, P, st0, rho);
    if (frac)
        for (int i = 0; i < I; i++) rho[3 * i] = frac[i];
    for (int n = 0; n < N; n++) {
        or_coarse_rho(pr, rho + n * RS, rho + (n + 1) * RS);
        memcpy(cache + n * RS, rho + (n + 1) * RS, sizeof(double) * RS);
        if (frac)
            for (int i = 0; i < I; i++) rho[(n + 1) * RS + 3 * i] = frac[(size_t)(n + 1) * I + i];
    }
    memcpy(cur, u0, sizeof(double) * P);
    for (int n = 1; n <= N; n++) {
        double *xn = cur + (size_t)n * P;
        memcpy(xn, u0, sizeof(double) * P);
        for (int i = 0; i < I; i++) {
            if (st0[i].n == 0)
                continue;
            double mu = rho[n * RS + 3 * i + 1], sig = rho[n * RS + 3 * i + 2];
            if (!(sig >= 0.0) || !isfinite(sig) || !isfinite(mu))
                continue;
            or_transform(pr, u0, xn, P, inst, n, i, &st0[i], mu, sig, 1);
        }
    }
    memcpy(rho_out, rho, sizeof(double) * (N + 1) * RS);
    for (int n = 0; n <= N; n++)
        or_rho_global(I, rho + n * RS, glob_out + 2 * n, glob_out + 2 * n + 1);
    if (states)
        memcpy(states, cur, sizeof(double) * (size_t)(N + 1) * P);

    int k;
    for (k = 0; k < K; k++) {
        /* fine propagator on the slices that are not yet exact (n >= k) */
        for (int n = k; n < N; n++) {
            memcpy(fine + (size_t)(n + 1) * P, cur + (size_t)n * P, sizeof(double) * P);
            or_fine(pr, fine + (size_t)(n + 1) * P, P, inst, n, NULL);
            or_restrict(pr, fine + (size_t)(n + 1) * P, P, rec + (size_t)(n + 1) * (I + 1));
        }

        /* learning: fit the fraction model to the slices that are exact after
           this fine sweep (n = 0..k+1), extrapolate beyond                    */
        double phat[257];
        int use_hat = 0;
        if (learning && I == 2) {
            double tt[257], yy[257];
            int npts = 0;
            for (int n = 0; n <= k + 1 && n <= N; n++) {
                tt[npts] = n * pr->dt * pr->steps_per_slice;
                yy[npts] = (n == 0) ? (double)st0[0].n / (double)P : (double)rec[(size_t)n * (I + 1)].n / (double)P;
                npts++;
            }
            if (npts >= 3) {
                double k0 = have_fit ? kappa : 1.0 / (N * pr->dt * pr->steps_per_slice);
                double p0 = have_fit ? pstar : yy[npts - 1];
                or_fraction_fit(npts, tt, yy, k0, p0, &kappa, &pstar);
                have_fit = 1;
            }
            if (have_fit) {
                use_hat = 1;
                double tk = (k + 1) * pr->dt * pr->steps_per_slice;
                double yk = yy[npts - 1];
                for (int n = 0; n <= N; n++) {
                    double tn = n * pr->dt * pr->steps_per_slice;
                    phat[n] = (n <= k + 1) ? -1.0 : pstar + (yk - pstar) * exp(-kappa * (tn - tk));
                }
            }
        }

        /* sequential coarse sweep with the iterator */
        memcpy(nrho, rho, sizeof(double) * RS); /* rho^{k+1}_0 = R(u0) */
        for (int n = 0; n < N; n++) {
            double a[24], *c = cache + n * RS;
            or_coarse_rho(pr, nrho + n * RS, a);
            memcpy(ncache + n * RS, a, sizeof(double) * RS);
            double *out = nrho + (n + 1) * RS;
            or_stats *b = rec + (size_t)(n + 1) * (I + 1);
            double *xb = fine + (size_t)(n + 1) * P;
            int32_t *fl = flags + ((size_t)k * N + n) * I;
            if (memcmp(a, c, sizeof(double) * RS) == 0) {
                /* I(a, b, a) = (R(b), b) */
                or_rho_from_stats(I, P, b, out);
                for (int i = 0; i < I; i++) fl[i] = 0;
                if (frac)
                    for (int i = 0; i < I; i++) out[3 * i] = frac[(size_t)(n + 1) * I + i];
                continue;
            }
            for (int i = 0; i < I; i++) {
                double fi = (double)b[i].n / (double)P;
                if (b[i].n == 0) {
                    out[3 * i] = 0.0;
                    out[3 * i + 1] = a[3 * i + 1];
                    out[3 * i + 2] = a[3 * i + 2];
                    fl[i] = 4;
                    continue;
                }
                double alM = (a[3 * i + 1] - c[3 * i + 1]) + b[i].mean;
                double alV = (a[3 * i + 2] - c[3 * i + 2]) + b[i].var;
                if (!(alV >= 0.0) || !isfinite(alV) || !isfinite(alM)) {
                    out[3 * i] = fi; out[3 * i + 1] = b[i].mean; out[3 * i + 2] = b[i].var;
                    fl[i] = 2;
                    continue;
                }
                int inside = or_transform(pr, xb, xb, P, inst, n + 1, i, &b[i], alM, alV, 0);
                if (!inside) {
                    out[3 * i] = fi; out[3 * i + 1] = b[i].mean; out[3 * i + 2] = b[i].var;
                    fl[i] = 3;
                    continue;
                }
                fl[i] = 1;
                out[3 * i] = fi; out[3 * i + 1] = alM; out[3 * i + 2] = alV;
            }
            /* move the accepted regions (decisions were taken on the
               unmoved ensemble; regions are disjoint and stay so)         */
            for (int i = 0; i < I; i++)
                if (fl[i] == 1) {
                    double alM = out[3 * i + 1], alV = out[3 * i + 2];
                    or_transform(pr, xb, xb, P, inst, n + 1, i, &b[i], alM, alV, 1);
                }
            /* learning: extrapolated fractions replace the fine fractions of
               slices beyond the exact ones in the macro state                */
            if (use_hat && phat[n + 1] >= 0.0) {
                out[0] = phat[n + 1];
                out[3] = 1.0 - phat[n + 1];
            }
            if (frac)
                for (int i = 0; i < I; i++) out[3 * i] = frac[(size_t)(n + 1) * I + i];
        }

        /* successive-iterate difference of the global moments */
        double d = 0.0;
        for (int n = 1; n <= N; n++) {
            double M0, V0, M1, V1;
            or_rho_global(I, rho + n * RS, &M0, &V0);
            or_rho_global(I, nrho + n * RS, &M1, &V1);
            if (fabs(M1 - M0) > d) d = fabs(M1 - M0);
            if (fabs(V1 - V0) > d) d = fabs(V1 - V0);
        }
        delta[k] = d;

        /* rotate: u^{k+1}_{n+1} = matched F(u^k_n) for n >= k; exact slices keep */
        for (int n = k; n < N; n++)
            memcpy(cur + (size_t)(n + 1) * P, fine + (size_t)(n + 1) * P, sizeof(double) * P);
        memcpy(rho, nrho, sizeof(double) * (N + 1) * RS);
        memcpy(cache, ncache, sizeof(double) * (N + 1) * RS);

        memcpy(rho_out + (size_t)(k + 1) * (N + 1) * RS, rho, sizeof(double) * (N + 1) * RS);
        for (int n = 0; n <= N; n++)
            or_rho_global(I, rho + n * RS, glob_out + (size_t)(k + 1) * (N + 1) * 2 + 2 * n,
                          glob_out + (size_t)(k + 1) * (N + 1) * 2 + 2 * n + 1);
        if (states)
            memcpy(states + (size_t)(k + 1) * (N + 1) * P, cur, sizeof(double) * (size_t)(N + 1) * P);
        if (d <= tol || k + 1 >= N) {
            k++;
            break;
        }
    }

    free(cur); free(fine); free(rho); free(nrho); free(cache); free(ncache); free(rec);
    return k;
}

/* ------------------------------------------------------------------------- */
/* Adjoint of the serial fine solution (discretise, then differentiate).      */
/*                                                                           */
/* J = sum_{n=1..N} (m_n - Mhat_n)^2 + (v_n - Vhat_n)^2, where (m_n, v_n) are */
/* the population moments at the end of slice n and the noise is fixed.      */
/* Returns J and dJ/dtheta for theta = (a0, a1, a2, a3, am, av, b0, b1, bm,  */
/* bv).  x: P initial particles (unchanged).  Straightforward: stores every  */
/* state of the forward solve (N*m + 1 states of P doubles).                  */
/* ------------------------------------------------------------------------- */
double or_adjoint(const or_problem *pr, const double *x0, int64_t P, uint32_t inst,
                  const double *Mhat, const double *Vhat, double *grad)
{
    if (pr->axs != 0.0 || or_is_trig(pr) || pr->wrap) /* terms not differentiated here */
        return NAN;
    int N = pr->n_slices, m = pr->steps_per_slice;
    int64_t S = (int64_t)N * m;
    double dt = pr->dt, sdt = sqrt(dt);
    double *X = (double *)malloc(sizeof(double) * (size_t)(S + 1) * P);
    double *mom = (double *)malloc(sizeof(double) * 2 * (size_t)(S + 1));
    double *lam = (double *)malloc(sizeof(double) * P);
    double *lnew = (double *)malloc(sizeof(double) * P);
    memcpy(X, x0, sizeof(double) * P);
    for (int64_t s = 0; s < S; s++) {
        const double *xs = X + (size_t)s * P;
        double *xn = X + (size_t)(s + 1) * P;
        or_moments(xs, P, &mom[2 * s], &mom[2 * s + 1]);
        double mj = mom[2 * s], vj = mom[2 * s + 1];
        for (int64_t p = 0; p < P; p++) {
            double z = or_normal_of(pr->seed, p, (uint32_t)s, inst, OR_TAG_EM);
            xn[p] = xs[p] + or_drift(pr, xs[p], mj, vj, 0.0, 0.0) * dt + or_diffusion(pr, xs[p], mj, vj) * sdt * z;
        }
    }
    or_moments(X + (size_t)S * P, P, &mom[2 * S], &mom[2 * S + 1]);

    double J = 0.0;
    for (int n = 1; n <= N; n++) {
        double em = mom[2 * (size_t)n * m] - Mhat[n - 1];
        double ev = mom[2 * (size_t)n * m + 1] - Vhat[n - 1];
        J += em * em + ev * ev;
    }
    for (int q = 0; q < 10; q++) grad[q] = 0.0;
    for (int64_t p = 0; p < P; p++) lam[p] = 0.0;

    /* lam_s = dJ/dX_s (total derivative through all later states) */
    for (int64_t s = S; s >= 0; s--) {
        const double *xs = X + (size_t)s * P;
        double ms = mom[2 * s], vs = mom[2 * s + 1];
        /* direct dependence of J on X_s when s is a slice end */
        if (s > 0 && s % m == 0) {
            int n = (int)(s / m);
            double em = ms - Mhat[n - 1], ev = vs - Vhat[n - 1];
            for (int64_t p = 0; p < P; p++)
                lam[p] += 2.0 * em / P + 2.0 * ev * 2.0 * (xs[p] - ms) / P;
        }
        if (s == 0)
            break;
        /* step s-1 -> s: X_s = X_{s-1} + a dt + b sdt z with (m, v) of X_{s-1} */
        const double *xp = X + (size_t)(s - 1) * P;
        double mp = mom[2 * (s - 1)], vp = mom[2 * (s - 1) + 1];
        double gm = 0.0, gv = 0.0; /* dJ/dm_{s-1}, dJ/dv_{s-1} through this step */
        for (int64_t p = 0; p < P; p++) {
            double z = or_normal_of(pr->seed, p, (uint32_t)(s - 1), inst, OR_TAG_EM);
            double x = xp[p], l = lam[p];
            gm += l * (pr->am * dt + pr->bm * sdt * z);
            gv += l * (pr->av * dt + pr->bv * sdt * z);
            grad[0] += l * dt;
            grad[1] += l * x * dt;
            grad[2] += l * x * x * dt;
            grad[3] += l * x * x * x * dt;
            grad[4] += l * mp * dt;
            grad[5] += l * vp * dt;
            grad[6] += l * sdt * z;
            grad[7] += l * x * sdt * z;
            grad[8] += l * mp * sdt * z;
            grad[9] += l * vp * sdt * z;
        }
        for (int64_t p = 0; p < P; p++) {
            double z = or_normal_of(pr->seed, p, (uint32_t)(s - 1), inst, OR_TAG_EM);
            double x = xp[p];
            double ax = pr->a1 + 2.0 * pr->a2 * x + 3.0 * pr->a3 * x * x;
            double bx = pr->b1;
            lnew[p] = lam[p] * (1.0 + ax * dt + bx * sdt * z) + gm / P + gv * 2.0 * (x - mp) / P;
        }
        memcpy(lam, lnew, sizeof(double) * P);
    }
    free(X); free(mom); free(lam); free(lnew);
    return J;
}
