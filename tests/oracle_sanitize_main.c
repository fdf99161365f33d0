/*
 * oracle_sanitize_main.c -- drives every entry point of the C oracle on
 * small cases, for a build with AddressSanitizer and UndefinedBehavior-
 * Sanitizer (tests/test_oracle.py builds it with gcc and runs it on the CPU).
 * The oracle is included as one translation unit, so its static helpers are
 * instrumented too.  Exit status 0 and no sanitizer report is the pass.
 */
#include "../oracle/mcpr_oracle.c"

#include <stdio.h>

static or_problem base_problem(void)
{
    or_problem pr;
    memset(&pr, 0, sizeof pr);
    pr.a1 = 0.5; /* Desai-Zwanzig double well with mean-field attraction */
    pr.a3 = -1.0;
    pr.am = 0.5;
    pr.b0 = 0.5;
    pr.p0_kind = 1;
    pr.p0_w = 0.5;
    pr.p0_mu1 = -1.0;
    pr.p0_sd1 = 0.1;
    pr.p0_mu2 = 1.0;
    pr.p0_sd2 = 0.1;
    pr.dt = 0.01;
    pr.steps_per_slice = 5;
    pr.n_slices = 6;
    pr.n_regions = 2;
    pr.coarse_substeps = 1;
    pr.split[0] = 0.0;
    pr.seed = 7;
    pr.coarse_model = 2;
    return pr;
}

int main(void)
{
    const int64_t P = 203; /* ragged: 50 quads and 3 particles */
    or_problem pr = base_problem();
    const int N = pr.n_slices, I = pr.n_regions, m = pr.steps_per_slice;
    double *x = (double *)malloc(sizeof(double) * P);
    double *y = (double *)malloc(sizeof(double) * P);
    double *F = (double *)malloc(sizeof(double) * P);
    double *trace = (double *)malloc(sizeof(double) * 2 * m);
    or_stats st[9];
    double sum = 0.0;

    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, w[4];
    or_philox4x32_10(ctr, key, w);
    double z[4];
    or_normals4(pr.seed, 0, 0, 0, 0, z);
    sum += or_uniform(w[0]) + z[0];

    or_sample_p0(&pr, P, 0, x);
    double mean, var;
    or_moments(x, P, &mean, &var);
    for (int kind = 0; kind < 3; kind++) sum += or_qoi(x, P, kind);
    sum += or_region_of(&pr, 0.25);
    or_restrict(&pr, x, P, st);
    or_fine(&pr, x, P, 0, 1, trace);
    or_empirical_cdf(x, P, F);
    double yin[4] = {-1.0, 0.02, 1.0, 0.03}, yout[4], f[2] = {0.4, 0.6};
    or_coarse(&pr, f, yin, yout);
    or_restrict(&pr, x, P, st);
    sum += or_transform(&pr, x, y, P, 0, 3, 1, &st[1], st[1].mean + 0.1, st[1].var * 1.2, 1);
    double rho[6] = {0.4, -1.0, 0.02, 0.6, 1.0, 0.03}, M, V;
    or_rho_global(I, rho, &M, &V);
    double t[5] = {0, 1, 2, 3, 4}, yy[5], kappa, pstar;
    for (int j = 0; j < 5; j++) yy[j] = 0.7 + (0.95 - 0.7) * exp(-0.3 * t[j]);
    or_fraction_fit(5, t, yy, 0.1, yy[4], &kappa, &pstar);

    /* serial solution and Parareal with learning and given fractions */
    or_stats *ser = (or_stats *)malloc(sizeof(or_stats) * (N + 1) * (I + 1));
    or_sample_p0(&pr, P, 0, x);
    memcpy(y, x, sizeof(double) * P);
    or_serial(&pr, y, P, 0, ser);
    const int K = 3;
    double *rho_out = (double *)malloc(sizeof(double) * (K + 1) * (N + 1) * I * 3);
    double *glob = (double *)malloc(sizeof(double) * (K + 1) * (N + 1) * 2);
    int32_t *flags = (int32_t *)malloc(sizeof(int32_t) * K * N * I);
    double *delta = (double *)malloc(sizeof(double) * K);
    double *states = (double *)malloc(sizeof(double) * (K + 1) * (N + 1) * P);
    double *frac = (double *)malloc(sizeof(double) * (N + 1) * I);
    for (int n = 0; n <= N; n++) {
        frac[n * I] = 0.5;
        frac[n * I + 1] = 0.5;
    }
    sum += or_parareal(&pr, x, P, 0, K, 0.0, 1, NULL, rho_out, glob, flags, delta, states);
    sum += or_parareal(&pr, x, P, 0, K, 1e-3, 0, frac, rho_out, glob, flags, delta, NULL);

    /* a point mass (resample branch) and the adjoint with every coefficient */
    or_problem pm = base_problem();
    pm.p0_kind = 2;
    pm.p0_mu1 = 0.5;
    pm.b0 = 0.0;
    or_sample_p0(&pm, P, 0, x);
    sum += or_parareal(&pm, x, P, 0, 2, 0.0, 0, NULL, rho_out, glob, flags, delta, NULL);
    or_problem pa = base_problem();
    pa.a0 = 0.05;
    pa.a2 = 0.05;
    pa.av = 0.2;
    pa.b1 = 0.02;
    pa.bm = 0.05;
    pa.bv = 0.1;
    double Mh[6] = {0.1, 0.1, 0.1, 0.1, 0.1, 0.1}, Vh[6] = {0.9, 0.9, 0.9, 0.9, 0.9, 0.9}, grad[10];
    or_sample_p0(&pa, P, 0, x);
    sum += or_adjoint(&pa, x, P, 0, Mh, Vh, grad);

    /* the rotator's trigonometric mean field with the wrap, and the Burgers drift */
    or_problem rot;
    memset(&rot, 0, sizeof rot);
    rot.ksin = -1.0;
    rot.kc = 1.0;
    rot.b0 = 1.0;
    rot.wrap = 1;
    rot.p0_kind = 0;
    rot.p0_mu1 = 0.785;
    rot.p0_sd1 = 1.5;
    rot.dt = 0.01;
    rot.steps_per_slice = 5;
    rot.n_slices = 4;
    rot.n_regions = 1;
    rot.coarse_substeps = 1;
    rot.coarse_model = 2;
    or_sample_p0(&rot, P, 0, x);
    sum += or_parareal(&rot, x, P, 0, 2, 0.0, 0, NULL, rho_out, glob, flags, delta, NULL);
    or_problem bu = rot;
    bu.ksin = bu.kc = 0.0;
    bu.wrap = 0;
    bu.acdf = 1.0;
    bu.p0_kind = 2;
    bu.p0_mu1 = 0.0;
    bu.coarse_model = 0;
    or_sample_p0(&bu, P, 0, x);
    or_fine(&bu, x, P, 0, 0, trace);

    printf("oracle entry points ran: %.6g\n", sum + mean + var + M + V + kappa + pstar + yout[0] + grad[0]);
    free(x);
    free(y);
    free(F);
    free(trace);
    free(ser);
    free(rho_out);
    free(glob);
    free(flags);
    free(delta);
    free(states);
    free(frac);
    return 0;
}
