"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  Each one ties a part of the oracle to
something other than the oracle itself: published known-answer vectors, exact
rational arithmetic, closed forms of the linear case (Lemma "Exactness of the
Taylor-based moment model for linear SDEs"), exact per-realisation identities of
the Euler-Maruyama recursion, the consistency lemma of S and T, the exactness
property of MC-moments Parareal, and statistics.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats as sps
from scipy.integrate import solve_ivp

from paper_2310_11365_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------- RNG
def test_philox_known_answer_vectors(oracle):
    """Philox4x32-10 reproduces the published known-answer vectors."""
    n = 0
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(t, 16) for t in line.split()]
        assert oracle.philox(w[0:4], w[4:6]) == w[6:10]
        n += 1
    assert n == 3


def test_uniform_map_is_exact(oracle):
    for w in [0, 1, 12345, 2**31, 2**32 - 1]:
        assert oracle.uniform(w) == (Fraction(w) + Fraction(1, 2)) / 2**32
    assert 0.0 < oracle.uniform(0) and oracle.uniform(2**32 - 1) < 1.0


def test_normals_statistics(oracle):
    """Box-Muller normals: mean 0, variance 1, KS against N(0,1)."""
    z = np.concatenate([oracle.normals4(7, q, 3, 1, 0) for q in range(25000)])
    assert abs(z.mean()) < 4.0 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 4.0 * math.sqrt(2.0 / z.size)
    assert sps.kstest(z, "norm").pvalue > 1e-3
    # the pairs of one call are uncorrelated
    zz = z.reshape(-1, 4)
    assert abs(np.corrcoef(zz[:, 0], zz[:, 1])[0, 1]) < 4.0 / math.sqrt(zz.shape[0])


def test_normals_depend_on_every_counter_word(oracle):
    base = oracle.normals4(0, 5, 6, 7, 0)
    for args in [(1, 5, 6, 7, 0), (0, 4, 6, 7, 0), (0, 5, 5, 7, 0), (0, 5, 6, 8, 0), (0, 5, 6, 7, 1)]:
        assert not np.array_equal(base, oracle.normals4(*args))


# --------------------------------------------------------------------------- moments / R
def _exact_moments(vals):
    fr = [Fraction(v) for v in vals]
    n = len(fr)
    m = sum(fr) / n
    v = sum((x - m) ** 2 for x in fr) / n
    return m, v


@pytest.mark.parametrize("P", [1, 2, 3, 5, 9])
def test_moments_match_exact_rationals(oracle, P):
    rng = np.random.default_rng(P)
    x = rng.normal(3.0, 2.0, P)
    m, v = oracle.moments(x)
    em, ev = _exact_moments(x)
    assert m == float(em)  # exact to the last bit for a few values
    assert abs(v - float(ev)) <= 1e-15 * max(1.0, float(ev))


def test_population_normalisation(oracle):
    """Weights 1/P: the empirical measure of the particle system, not 1/(P-1)."""
    m, v = oracle.moments(np.array([0.0, 2.0]))
    assert (m, v) == (1.0, 1.0)


def test_restriction_regions_ties_empty_degenerate(oracle):
    pr = W.dz_bimodal(P=8).problem
    x = np.array([-2.0, -1.0, 0.0, 1.0, 3.0, -0.5, 0.0, 2.0])
    st = oracle.restrict(pr, x)
    left, right, glob = st[0], st[1], st[2]
    assert left["n"] == 3 and right["n"] == 5 and glob["n"] == 8  # ties at 0 go to the upper region
    em, ev = _exact_moments([-2.0, -1.0, -0.5])
    assert abs(left["mean"] - float(em)) < 1e-15 and abs(left["var"] - float(ev)) < 1e-15
    assert left["min"] == -2.0 and left["max"] == -0.5
    # mixture formula equals the direct global moments
    f = np.array([left["n"], right["n"]]) / 8.0
    M = f[0] * left["mean"] + f[1] * right["mean"]
    V = f[0] * (left["var"] + (left["mean"] - M) ** 2) + f[1] * (right["var"] + (right["mean"] - M) ** 2)
    assert abs(M - glob["mean"]) < 1e-15 and abs(V - glob["var"]) < 1e-14
    rho = np.array([f[0], left["mean"], left["var"], f[1], right["mean"], right["var"]])
    gM, gV = oracle.rho_global(rho)
    assert abs(gM - glob["mean"]) < 1e-15 and abs(gV - glob["var"]) < 1e-14
    # empty region
    st = oracle.restrict(pr, np.array([1.0, 2.0]))
    assert st[0]["n"] == 0 and st[0]["mean"] == 0.0 and st[0]["var"] == 0.0
    # all particles equal: variance exactly zero, mean exactly the value
    st = oracle.restrict(pr, np.full(7, 0.1))
    assert st[1]["n"] == 7 and st[1]["mean"] == 0.1 and st[1]["var"] == 0.0


def test_mixture_identity_random(oracle):
    pr = W.dz_bimodal(P=1000).problem
    x = oracle.sample_p0(pr, 1000)
    st = oracle.restrict(pr, x)
    rho = np.array([[s["n"] / 1000.0, s["mean"], s["var"]] for s in st[:2]]).ravel()
    gM, gV = oracle.rho_global(rho)
    assert abs(gM - st[2]["mean"]) < 1e-14
    assert abs(gV - st[2]["var"]) < 1e-13 * st[2]["var"]


# --------------------------------------------------------------------------- QoI
def test_qoi_exact_values(oracle):
    """(1/P) sum Phi: sin(0) = 0 and sin(pi/2) = 1 give exactly 1/2; x and x^2
    against exact rationals."""
    assert oracle.qoi(np.array([0.0, math.sqrt(math.pi / 2)]), oracle.QOI_SIN_X2) == 0.5
    x = np.array([0.5, -1.25, 3.0, 0.125])
    fr = [Fraction(v) for v in x]
    assert oracle.qoi(x, oracle.QOI_X) == float(sum(fr) / 4)
    assert oracle.qoi(x, oracle.QOI_X2) == float(sum(v * v for v in fr) / 4)


def test_qoi_sin_x2_gaussian_closed_form(oracle):
    """For X ~ N(mu, s^2), E[exp(i X^2)] = (1 - 2 i s^2)^(-1/2) exp(i mu^2 / (1 - 2 i s^2)),
    so E[sin X^2] is its imaginary part (mu = 1, s = 1/2: the GBM example's p0)."""
    import cmath
    pr = W.gbm().problem
    x = oracle.sample_p0(pr, 400_000)
    z = 1 - 2j * 0.25
    exact = (cmath.exp(1j / z) / cmath.sqrt(z)).imag
    se = np.sin(x * x).std() / math.sqrt(x.size)
    assert abs(oracle.qoi(x, oracle.QOI_SIN_X2) - exact) < 4 * se


# --------------------------------------------------------------------------- p0
def test_initial_law_sample_moments(oracle):
    pr = W.ou_linear().problem
    x = oracle.sample_p0(pr, 40000)
    assert abs(x.mean() - 1.0) < 4 * 0.2 / 200
    assert abs(x.std() - 0.2) < 4 * 0.2 / math.sqrt(2 * 40000)
    pr = W.dz_bimodal().problem
    x = oracle.sample_p0(pr, 40000)
    frac_left = np.mean(x < 0)
    assert abs(frac_left - 0.5) < 4 * 0.5 / 200
    assert abs(x[x < 0].mean() + 1.0) < 0.01 and abs(x[x >= 0].std() - 0.1) < 0.01
    pr.p0 = W.P0(W.P0_DELTA, mu1=100.0)
    assert np.all(oracle.sample_p0(pr, 10) == 100.0)


# --------------------------------------------------------------------------- EM
def test_em_deterministic_closed_form(oracle):
    """sigma = 0, P = 1: the mean field is the particle itself, and the scheme
    is explicit Euler for x' = (a1 + am) x + a0."""
    pr = W.make_problem(W.Coef(a0=0.3, a1=-1.0, am=0.5), W.P0(W.P0_DELTA, mu1=2.0), 1.0, 10, 1e-3)
    x, _ = oracle.fine(pr, np.array([2.0]), 0)
    lam, c = -0.5, 0.3
    expect = 2.0
    for _ in range(pr.steps_per_slice):
        expect = expect + (lam * expect + c) * pr.dt
    assert abs(x[0] - expect) < 1e-14
    closed = (1 + lam * pr.dt) ** 100 * (2.0 + c / lam) - c / lam
    assert abs(x[0] - closed) < 1e-13


def _em_normals(oracle, pr, P, s, inst=0):
    q = (P + 3) // 4
    return np.concatenate([oracle.normals4(pr.seed, i, s, inst, 0) for i in range(q)])[:P]


@pytest.mark.parametrize("slice_index", [0, 3])
def test_em_per_realisation_identities(oracle, slice_index):
    """Linear drift, additive noise: for any P the EM moments obey
      M_{j+1} = (1 + (a1+am) dt) M_j + a0 dt + b0 sqrt(dt) mean(z_j)
      V_{j+1} = (1 + a1 dt)^2 V_j + 2 (1 + a1 dt) b0 sqrt(dt) Cov(X_j, z_j) + b0^2 dt Var(z_j)
    with the normals drawn at global step s = n m + j."""
    pr = W.make_problem(W.Coef(a0=0.2, a1=-1.0, am=0.5, b0=0.3), W.P0(W.P0_NORMAL, 1, 1.0, 0.2),
                        1.0, 10, 1e-2)
    P = 37
    x0 = oracle.sample_p0(pr, P)
    x1, tr = oracle.fine(pr, x0, slice_index, trace=True)
    X = x0.copy()
    a1, am, a0, b0, dt = -1.0, 0.5, 0.2, 0.3, pr.dt
    for j in range(pr.steps_per_slice):
        z = _em_normals(oracle, pr, P, slice_index * pr.steps_per_slice + j)
        M, V = X.mean(), X.var()
        assert abs(tr[j, 0] - M) < 1e-14 and abs(tr[j, 1] - V) < 1e-14
        Mn = (1 + (a1 + am) * dt) * M + a0 * dt + b0 * math.sqrt(dt) * z.mean()
        cov = np.mean((X - M) * (z - z.mean()))
        Vn = (1 + a1 * dt) ** 2 * V + 2 * (1 + a1 * dt) * b0 * math.sqrt(dt) * cov + b0 ** 2 * dt * z.var()
        X = X + (a1 * X + am * M + a0) * dt + b0 * math.sqrt(dt) * z
        assert abs(X.mean() - Mn) < 1e-13 and abs(X.var() - Vn) < 1e-13
    np.testing.assert_allclose(x1, X, rtol=0, atol=1e-13)


def test_em_nonlinear_bruteforce(oracle):
    """Tiny ensemble, full coefficient set (cubic drift, multiplicative and
    mean-field diffusion, variance dependence, the x E[X^2] term): step by
    step against a direct evaluation with exact rational arithmetic of each
    step's moments."""
    coef = W.Coef(a0=0.1, a1=0.5, a2=-0.2, a3=-1.0, am=0.5, av=0.3, b0=0.4, b1=0.1, bm=-0.05, bv=0.2, axs=-0.3)
    pr = W.make_problem(coef, W.P0(W.P0_MIXTURE, 0.5, -1.0, 0.1, 1.0, 0.1), 0.05, 5, 1e-3, (0.0,))
    P = 6
    x0 = oracle.sample_p0(pr, P)
    x1, _ = oracle.fine(pr, x0, 2)
    X = [float(v) for v in x0]
    for j in range(pr.steps_per_slice):
        z = _em_normals(oracle, pr, P, 2 * pr.steps_per_slice + j)
        M, V = _exact_moments(X)
        M, V = float(M), float(V)
        new = []
        for p in range(P):
            x = X[p]
            a = (coef.a0 + coef.a1 * x + coef.a2 * x * x + coef.a3 * x ** 3 + coef.am * M + coef.av * V
                 + coef.axs * x * (V + M * M))
            b = coef.b0 + coef.b1 * x + coef.bm * M + coef.bv * V
            new.append(x + a * pr.dt + b * math.sqrt(pr.dt) * z[p])
        X = new
    np.testing.assert_allclose(x1, X, rtol=0, atol=1e-13)


def test_em_statistics_match_ou_closed_form(oracle):
    """Linear mean-field OU of the base workload: conditional on the realised
    initial moments, E[M_n] = (1 - 0.5 dt)^n M_0 and
    E[V_{n+1}] = (1 - dt)^2 E[V_n] + 0.09 dt (P-1)/P.  z-scores < 5."""
    wl = W.ou_linear(P=10_000, N=1)
    pr = wl.problem
    pr.steps_per_slice = 300
    x0 = oracle.sample_p0(pr, wl.P)
    m0, v0 = oracle.moments(x0)
    x1, _ = oracle.fine(pr, x0, 0)
    m1, v1 = oracle.moments(x1)
    n, dt, P = pr.steps_per_slice, pr.dt, wl.P
    EM = (1 - 0.5 * dt) ** n * m0
    EV = v0
    for _ in range(n):
        EV = (1 - dt) ** 2 * EV + 0.09 * dt * (P - 1) / P
    t = n * dt
    se_m = math.sqrt(0.09 * (1 - math.exp(-2 * t)) / 2 / P)
    se_v = math.sqrt(2.0 / P) * EV
    assert abs(m1 - EM) < 5 * se_m
    assert abs(v1 - EV) < 5 * se_v


# --------------------------------------------------------------------------- coarse
def test_rk4_affine_closed_form(oracle):
    """OU workload: the moment model is dM/dt = -0.5 M, dV/dt = -2 V + 0.09; RK4
    on an affine ODE y' = l y + c is y <- R(h l)(y + c/l) - c/l with
    R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24."""
    pr = W.ou_linear().problem
    h = pr.slice_length / pr.coarse_substeps
    R = lambda z: 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    assert R(-0.025) == pytest.approx(0.975309912109375, abs=1e-16)
    y = np.array([1.0, 0.04])
    M, V = 1.0, 0.04
    for _ in range(pr.n_slices):
        y = oracle.coarse(pr, [1.0], y)
        for _ in range(pr.coarse_substeps):
            M = R(-0.5 * h) * M
            V = R(-2.0 * h) * (V - 0.045) + 0.045
        assert abs(y[0] - M) < 1e-14 and abs(y[1] - V) < 1e-14
    # and the continuous solution to RK4 accuracy
    assert abs(y[0] - math.exp(-0.5)) < 1e-8
    assert abs(y[1] - (0.045 - 0.005 * math.exp(-2.0))) < 1e-8


def test_coarse_linear_lemma(oracle):
    """For linear coefficients the Taylor model is exact:
    dM/dt = (a1 + am) M + a0,  dV/dt = (2 a1 + b1^2) V + (b0 + (b1 + bm) M)^2."""
    coef = W.Coef(a0=0.3, a1=-0.8, am=0.4, b0=0.2, b1=0.3, bm=0.1)
    pr = W.make_problem(coef, W.P0(), 1.0, 4, 1e-3, coarse_h=0.001)
    y0 = np.array([1.5, 0.2])
    y = oracle.coarse(pr, [1.0], y0)

    def rhs(t, u):
        M, V = u
        return [(coef.a1 + coef.am) * M + coef.a0,
                (2 * coef.a1 + coef.b1 ** 2) * V + (coef.b0 + (coef.b1 + coef.bm) * M) ** 2]
    sol = solve_ivp(rhs, (0, pr.slice_length), y0, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(y, sol.y[:, -1], rtol=1e-11)


def test_coarse_polynomial_drift_is_exact_moment_ode(oracle):
    """dX = (alpha X + E[X] - X E[X^2]) dt + X dW (the polynomial-drift example
    of the appendix on the exactness of the moment model): the Taylor model is
    the known exact moment system dM = (alpha + 1) M - M S,
    dS = (2 alpha + 1) S + 2 M^2 - 2 S^2 with S = E[X^2].  The oracle's RK4
    (h = 0.05) against a tight solve of that system, in (M, Sigma = S - M^2)."""
    alpha = 0.5
    wl = W.polydrift(alpha=alpha, N=10, T=2.0)
    pr = wl.problem
    y0 = np.array([1.0, 0.0])  # X(0) = 1
    y = y0.copy()
    ts = [0.0]
    ys = [y.copy()]
    for n in range(pr.n_slices):
        y = oracle.coarse(pr, np.array([1.0]), y)
        ys.append(y.copy())
        ts.append((n + 1) * pr.slice_length)

    def rhs(t, u):
        M, S = u
        return [(alpha + 1) * M - M * S, (2 * alpha + 1) * S + 2 * M * M - 2 * S * S]
    sol = solve_ivp(rhs, (0.0, ts[-1]), [1.0, 1.0], t_eval=ts, rtol=1e-12, atol=1e-14)
    for n in range(1, len(ts)):
        M, S = sol.y[0, n], sol.y[1, n]
        assert abs(ys[n][0] - M) < 1e-6 and abs(ys[n][1] - (S - M * M)) < 1e-6, n


def test_rotator_em_bruteforce_pair_sum(oracle):
    """Plane rotator, tiny ensemble: every step against the direct pair sum
    (K/P) sum_q sin(X_q - X_p) - sin X_p, unit noise, and the shift modulo
    2 pi into [0, 2 pi); the trace holds the means of sin X and cos X."""
    wl = W.rotator(P=5, N=4, T=0.2, dt=1e-2)
    pr = wl.problem
    c = pr.coef
    x0 = oracle.sample_p0(pr, 5)
    x1, tr = oracle.fine(pr, x0, 1, trace=True)
    X = x0.copy()
    two_pi = 6.283185307179586
    for j in range(pr.steps_per_slice):
        z = _em_normals(oracle, pr, 5, pr.steps_per_slice + j)
        assert abs(tr[j, 0] - np.mean(np.sin(X))) < 1e-15 and abs(tr[j, 1] - np.mean(np.cos(X))) < 1e-15
        pair = np.array([np.mean(np.sin(X - xp)) for xp in X])
        X = X + (c.kc * pair + c.ksin * np.sin(X)) * pr.dt + c.b0 * math.sqrt(pr.dt) * z
        X = X - two_pi * np.floor(X / two_pi)
    np.testing.assert_allclose(x1, X, rtol=0, atol=1e-13)
    assert np.all((x1 >= 0) & (x1 < two_pi))


def test_rotator_taylor_model_is_the_printed_one(oracle):
    """One region: the Taylor model of the plane rotator is dM = -sin M +
    (Sigma/2) sin M, dSigma = 2 (-K - cos M) Sigma + 2 kB T (the paper's model,
    read with a_x = -K - cos M); the oracle's RK4 against a tight solve."""
    K, kT = 1.3, 0.4
    wl = W.rotator(K=K, kT=kT, N=10, T=2.0)
    pr = wl.problem
    y = np.array([math.pi / 4, 0.3])
    ys, ts = [y.copy()], [0.0]
    for n in range(pr.n_slices):
        y = oracle.coarse(pr, np.array([1.0]), y)
        ys.append(y.copy())
        ts.append((n + 1) * pr.slice_length)

    def rhs(t, u):
        M, S = u
        return [-math.sin(M) + 0.5 * S * math.sin(M), 2 * (-K - math.cos(M)) * S + 2 * kT]
    sol = solve_ivp(rhs, (0.0, ts[-1]), ys[0], t_eval=ts, rtol=1e-12, atol=1e-14)
    for n in range(1, len(ts)):
        assert np.max(np.abs(ys[n] - sol.y[:, n])) < 1e-6, n
    # without noise a point mass stays one, the sigma points collapse, and the
    # Gaussian models coincide with the Taylor model (M' = -sin M)
    pr0 = W.rotator(K=K, kT=0.0, N=10, T=2.0).problem
    t = oracle.coarse(pr0, np.array([1.0]), np.array([0.7, 0.0]))
    for model in (W.COARSE_GAUSS2, W.COARSE_GAUSS3):
        pr0.coarse_model = model
        g = oracle.coarse(pr0, np.array([1.0]), np.array([0.7, 0.0]))
        assert abs(g[0] - t[0]) < 1e-14 and g[1] == 0.0 and t[1] == 0.0


def test_empirical_cdf_bruteforce_with_ties(oracle):
    """F[p] = (1/P) sum_q H(x_p - x_q) with H(0) = 1/2, ties included, against
    the direct double sum."""
    rng = np.random.default_rng(4)
    x = np.round(rng.normal(0.0, 1.0, 301), 1)  # many ties
    H = lambda d: np.where(d > 0, 1.0, np.where(d == 0, 0.5, 0.0))
    direct = np.array([H(xp - x).sum() for xp in x]) / x.size
    np.testing.assert_array_equal(oracle.empirical_cdf(x), direct)
    assert np.all(oracle.empirical_cdf(np.zeros(8)) == 0.5)  # a point mass


def test_burgers_mean_moves_at_speed_half(oracle):
    """sum_p F_P(x_p) = P/2 for every configuration, so each Euler-Maruyama step
    moves the ensemble mean by exactly dt/2 + sigma sqrt(dt) mean(z) (the
    travelling wave of speed 1/2), from the point mass on."""
    wl = W.burgers(P=257, N=4, T=0.2, dt=1e-2, sigma=0.7)
    pr = wl.problem
    x0 = oracle.sample_p0(pr, wl.P)
    _, tr = oracle.fine(pr, x0, 1, trace=True)
    x1, _ = oracle.fine(pr, x0.copy(), 1)
    m_end = x1.mean()
    ms = list(tr[:, 0]) + [m_end]
    for j in range(pr.steps_per_slice):
        z = _em_normals(oracle, pr, wl.P, pr.steps_per_slice + j)
        assert abs(ms[j + 1] - ms[j] - 0.5 * pr.dt - 0.7 * math.sqrt(pr.dt) * z.mean()) < 1e-14, j


def test_burgers_moment_model(oracle):
    """The Taylor model with the Gaussian-density closure of the CDF term is
    the printed Burgers model dM = 1/2, dSigma = -(2/sqrt(2 pi)) sqrt(Sigma) + sigma^2."""
    sigma = 0.8
    pr = W.burgers(sigma=sigma, N=10, T=2.0).problem
    rhs = lambda t, u: [0.5, -2.0 / math.sqrt(2 * math.pi) * math.sqrt(max(u[1], 0.0)) + sigma ** 2]
    # from a spread state the RK4 coarse solver follows the model closely; from
    # the point mass sqrt(Sigma) is not smooth at 0 and RK4 is less accurate
    for y0, tol in ((np.array([0.3, 0.3]), 1e-7), (np.array([0.0, 0.0]), 3e-4)):
        y = y0.copy()
        ys, ts = [y.copy()], [0.0]
        for n in range(pr.n_slices):
            y = oracle.coarse(pr, np.array([1.0]), y)
            ys.append(y.copy())
            ts.append((n + 1) * pr.slice_length)
        sol = solve_ivp(rhs, (0.0, ts[-1]), y0, t_eval=ts, rtol=1e-12, atol=1e-14)
        for n in range(1, len(ts)):
            assert abs(ys[n][0] - sol.y[0, n]) < 1e-12 and abs(ys[n][1] - sol.y[1, n]) < tol, (y0, n)


def test_coarse_nonlinear_model_terms(oracle):
    """Double well: dM_i = a(M_i, mbar) + a_xx(M_i) V_i / 2 and
    dV_i = 2 a_x(M_i) V_i + b^2, regions coupled through the mixture mean."""
    pr = W.make_problem(W.dz_coef(), W.P0(), 0.1, 1, 1e-3, (0.0,), coarse_h=1e-4)
    f = np.array([0.3, 0.7])
    y0 = np.array([-1.0, 0.02, 0.9, 0.05])

    def rhs(t, u):
        M = u[0::2]
        V = u[1::2]
        mbar = f @ M
        out = []
        for i in range(2):
            a = 0.5 * M[i] - M[i] ** 3 + 0.5 * mbar
            out += [a - 3.0 * M[i] * V[i], 2 * (0.5 - 3 * M[i] ** 2) * V[i] + 0.25]
        return out
    sol = solve_ivp(rhs, (0, pr.slice_length), y0, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(oracle.coarse(pr, f, y0), sol.y[:, -1], rtol=1e-10)


def test_coarse_multimodal_equivalent_for_linear(oracle):
    """Property: for linear SDEs the per-region model with constant weights,
    recombined by the mixture formula, equals the unimodal model (to RK4
    accuracy)."""
    coef = W.Coef(a0=0.1, a1=-0.7, am=0.3, b0=0.3, b1=0.2, bm=0.05)
    pr2 = W.make_problem(coef, W.P0(), 0.5, 1, 1e-3, (0.0,), coarse_h=1e-3)
    pr1 = W.make_problem(coef, W.P0(), 0.5, 1, 1e-3, (), coarse_h=1e-3)
    f = np.array([0.4, 0.6])
    y = np.array([-1.0, 0.1, 1.2, 0.05])
    y2 = oracle.coarse(pr2, f, y)
    rho0 = np.array([f[0], y[0], y[1], f[1], y[2], y[3]])
    M0, V0 = oracle.rho_global(rho0)
    y1 = oracle.coarse(pr1, [1.0], [M0, V0])
    M2, V2 = oracle.rho_global(np.array([f[0], y2[0], y2[1], f[1], y2[2], y2[3]]))
    assert abs(M2 - y1[0]) < 1e-11 and abs(V2 - y1[1]) < 1e-11


@pytest.mark.parametrize("model", [W.COARSE_GAUSS2, W.COARSE_GAUSS3])
def test_gaussian_model_equals_taylor_for_linear(oracle, model):
    """For linear coefficients every Gaussian closure is exact and equals the
    Taylor model (Lemma on exactness for linear SDEs)."""
    coef = W.Coef(a0=0.3, a1=-0.8, am=0.4, av=0.1, b0=0.2, b1=0.3, bm=0.1, bv=0.05)
    pt = W.make_problem(coef, W.P0(), 0.5, 1, 1e-3, (0.0,), coarse_h=0.01)
    pg = W.make_problem(coef, W.P0(), 0.5, 1, 1e-3, (0.0,), coarse_h=0.01)
    pg.coarse_model = model
    f = np.array([0.35, 0.65])
    y = np.array([-0.7, 0.05, 1.1, 0.02])
    np.testing.assert_allclose(oracle.coarse(pg, f, y), oracle.coarse(pt, f, y), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("model,c4", [(W.COARSE_GAUSS2, 1.0), (W.COARSE_GAUSS3, 3.0)])
def test_gaussian_model_closed_form_cubic(oracle, model, c4):
    """Cubic drift, affine diffusion, x ~ N(M, V):
    E[a] = a0 + a1 M + a2 (M^2 + V) + a3 (M^3 + 3 M V) + am mbar + av vbar,
    E[(x - M) a] = a1 V + 2 a2 M V + a3 (3 M^2 V + c4 V^2),
    E[b^2] = (b0 + b1 M + bm mbar + bv vbar)^2 + b1^2 V,
    with c4 = 3 (exact Gaussian fourth moment, three sigma points) or
    c4 = 1 (two sigma points M +- sqrt(V))."""
    c = W.Coef(a0=0.1, a1=0.5, a2=-0.2, a3=-1.0, am=0.5, av=0.3, b0=0.4, b1=0.1, bm=-0.05, bv=0.2)
    pr = W.make_problem(c, W.P0(), 0.1, 1, 1e-3, (0.0,), coarse_h=1e-4)
    pr.coarse_model = model
    f = np.array([0.3, 0.7])
    y0 = np.array([-1.0, 0.02, 0.9, 0.05])

    def rhs(t, u):
        M, V = u[0::2], u[1::2]
        mbar = f @ M
        vbar = f @ (V + (M - mbar) ** 2)
        out = []
        for i in range(2):
            m, v = M[i], V[i]
            ea = c.a0 + c.a1 * m + c.a2 * (m * m + v) + c.a3 * (m ** 3 + 3 * m * v) + c.am * mbar + c.av * vbar
            exa = c.a1 * v + 2 * c.a2 * m * v + c.a3 * (3 * m * m * v + c4 * v * v)
            eb2 = (c.b0 + c.b1 * m + c.bm * mbar + c.bv * vbar) ** 2 + c.b1 ** 2 * v
            out += [ea, 2 * exa + eb2]
        return out
    sol = solve_ivp(rhs, (0, pr.slice_length), y0, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(oracle.coarse(pr, f, y0), sol.y[:, -1], rtol=1e-10)


def test_gaussian_model_stable_for_large_bimodal(oracle):
    """The large bimodal workload's coarse trajectory stays finite with the
    three-point Gaussian model over T = 10; the Taylor model's diverges."""
    wl = W.dz_large()
    y = np.array([-1.0, 0.01, 1.0, 0.01])
    f = np.array([0.5, 0.5])
    yt = y.copy()
    pt = W.dz_large().problem
    pt.coarse_model = W.COARSE_TAYLOR
    for _ in range(wl.problem.n_slices):
        y = oracle.coarse(wl.problem, f, y)
        with np.errstate(all="ignore"):
            yt = oracle.coarse(pt, f, yt)
    assert np.all(np.isfinite(y)) and np.all(y[1::2] > 0) and np.all(y[1::2] < 1)
    assert not np.all(np.isfinite(yt)) or np.max(np.abs(yt)) > 1e3


def test_coarse_matches_particles_for_linear(oracle):
    """The exact moment model and the particle system agree to within the MC
    error plus the O(dt) bias of EM."""
    wl = W.ou_linear(P=20000, N=2)
    pr = wl.problem
    x0 = oracle.sample_p0(pr, wl.P)
    m0, v0 = oracle.moments(x0)
    x1, _ = oracle.fine(pr, x0, 0)
    m1, v1 = oracle.moments(x1)
    y = oracle.coarse(pr, [1.0], [m0, v0])
    assert abs(m1 - y[0]) < 5 * math.sqrt(0.09 * 0.1 / wl.P) + 1e-4
    assert abs(v1 - y[1]) < 5 * math.sqrt(2.0 / wl.P) * y[1] + 1e-4


# --------------------------------------------------------------------------- matching
def test_transform_consistency_lemma(oracle):
    """S(T(rho, u)) = rho (Lemma on consistency of S and T) and T(S(u), u) = u."""
    pr = W.ou_linear().problem
    x = oracle.sample_p0(pr, 5000)
    st = oracle.restrict(pr, x)
    y, inside = oracle.transform(pr, x, 0, st[0], 0.37, 0.0123)
    assert inside
    m, v = oracle.moments(y)
    assert abs(m - 0.37) < 1e-14 and abs(v - 0.0123) < 1e-14 * 0.0123 * 50
    y, _ = oracle.transform(pr, x, 0, st[0], st[0]["mean"], st[0]["var"])
    np.testing.assert_allclose(y, x, rtol=0, atol=1e-15)


def test_transform_degenerate_branch(oracle):
    """V[u] = 0 (point mass, the perturbed-OU example's initial condition):
    T resamples sqrt(sigma) xi + mu with the matching normals."""
    pr = W.ou_linear().problem
    x = np.full(4000, 100.0)
    st = oracle.restrict(pr, x)
    assert st[0]["var"] == 0.0
    y, inside = oracle.transform(pr, x, 0, st[0], 99.0, 0.25, boundary=3)
    assert inside
    z = np.concatenate([oracle.normals4(pr.seed, q, 3, 0, 3) for q in range(1000)])
    np.testing.assert_allclose(y, 0.5 * z + 99.0, rtol=0, atol=1e-13)


def test_transform_acceptance_is_per_particle(oracle):
    """The in-region check of the multimodal iterator is exact particle by
    particle."""
    pr = W.dz_bimodal(P=2000).problem
    x = oracle.sample_p0(pr, 2000)
    st = oracle.restrict(pr, x)
    for mu, sig in [(1.0, 0.01), (0.5, 0.04), (0.2, 0.04), (1.0, 0.3)]:
        y, inside = oracle.transform(pr, x, 1, st[1], mu, sig, apply=True)
        moved = x >= 0
        assert inside == bool(np.all(y[moved] >= 0.0))
        np.testing.assert_array_equal(y[~moved], x[~moved])


# --------------------------------------------------------------------------- driver
def _invariant_check(oracle, wl, K, exact_fractions=False, learning=False):
    pr = wl.problem
    u0 = oracle.sample_p0(pr, wl.P)
    xs, st_serial = oracle.serial(pr, u0)
    fr = None
    if exact_fractions:
        fr = st_serial[:, :pr.n_regions]["n"] / wl.P
    res = oracle.parareal(pr, u0, K, keep_states=True, fractions=fr, learning=learning)
    # serial states, slice by slice
    ser = [u0.copy()]
    x = u0.copy()
    for n in range(pr.n_slices):
        x, _ = oracle.fine(pr, x, n)
        ser.append(x)
    I = pr.n_regions
    for k in range(res["iterations"] + 1):
        for n in range(0, min(k, pr.n_slices) + 1):
            assert np.array_equal(res["states"][k, n], ser[n]), (k, n)
            for i in range(I):
                assert res["rho"][k, n, i, 0] == st_serial[n, i]["n"] / wl.P
                assert res["rho"][k, n, i, 1] == st_serial[n, i]["mean"]
                assert res["rho"][k, n, i, 2] == st_serial[n, i]["var"]
    return res, st_serial


def test_parareal_exactness_unimodal(oracle):
    """Property (exactness of MC-moments Parareal): with the same random
    numbers in every iteration, u^k_n = u_n and rho^k_n = R(u_n) for n <= k,
    bit for bit."""
    wl = W.ou_linear(P=500, N=6)
    res, st = _invariant_check(oracle, wl, 6)
    assert res["iterations"] == 6
    # after N iterations the whole trajectory is the serial one
    np.testing.assert_array_equal(res["glob"][-1, :, 0], [s["mean"] for s in st[:, -1]])


def test_parareal_exactness_bimodal(oracle):
    wl = W.dz_bimodal(P=800, N=6)
    res, st = _invariant_check(oracle, wl, 6)
    fl = res["flags"]
    for k in range(fl.shape[0]):
        assert np.all(fl[k, :k + 1] == 0)  # exact slices take the I(a,b,a) branch


def test_parareal_exact_fractions_variant(oracle):
    """Reference variant with the serial solution's particle fractions (the
    exact-fraction variant of Sec. 5.3): exactness still holds bit for bit,
    every macro state carries the given fractions at every iteration, and the
    first iterate differs from the plain variant's (the fractions enter the
    coarse model's mean-field arguments)."""
    wl = W.dz_bimodal(P=800, N=6)
    res, st = _invariant_check(oracle, wl, 6, exact_fractions=True)
    fr = st[:, :2]["n"] / wl.P
    for k in range(res["iterations"] + 1):
        np.testing.assert_array_equal(res["rho"][k, :, :, 0], fr)
    u0 = oracle.sample_p0(wl.problem, wl.P)
    plain = oracle.parareal(wl.problem, u0, 2)
    assert not np.array_equal(plain["glob"][1], res["glob"][1])


def test_parareal_given_fractions_unimodal_is_plain(oracle):
    """With one region every fraction is 1: giving them changes nothing, bit for bit."""
    wl = W.ou_linear(P=500, N=5)
    pr = wl.problem
    u0 = oracle.sample_p0(pr, wl.P)
    a = oracle.parareal(pr, u0, 3, keep_states=True)
    b = oracle.parareal(pr, u0, 3, keep_states=True, fractions=np.ones((pr.n_slices + 1, 1)))
    for key in ("rho", "glob", "flags", "delta", "states"):
        np.testing.assert_array_equal(a[key], b[key])


def test_parareal_linear_converges_fast(oracle):
    """The coarse model is exact for the linear case, so after one iteration
    the Parareal moments are within the MC/time-step error of the serial run."""
    wl = W.ou_linear(P=4000, N=10)
    pr = wl.problem
    u0 = oracle.sample_p0(pr, wl.P)
    _, st = oracle.serial(pr, u0)
    res = oracle.parareal(pr, u0, 3)
    ser_m = np.array([s["mean"] for s in st[:, -1]])
    ser_v = np.array([s["var"] for s in st[:, -1]])
    e_mean = [np.max(np.abs(res["glob"][k, :, 0] - ser_m)) for k in range(res["iterations"] + 1)]
    e_var = [np.max(np.abs(res["glob"][k, :, 1] - ser_v)) for k in range(res["iterations"] + 1)]
    assert e_mean[1] < e_mean[0] or e_mean[0] < 1e-3
    assert e_mean[1] < 5e-3 and e_var[1] < 5e-3
    assert res["flags"][0, 1:, 0].tolist().count(1) >= 8  # matched, not rejected


def test_parareal_global_is_mixture(oracle):
    wl = W.dz_bimodal(P=600, N=4)
    pr = wl.problem
    u0 = oracle.sample_p0(pr, wl.P)
    res = oracle.parareal(pr, u0, 2)
    for k in range(res["iterations"] + 1):
        for n in range(pr.n_slices + 1):
            M, V = oracle.rho_global(res["rho"][k, n].ravel())
            assert res["glob"][k, n, 0] == M and res["glob"][k, n, 1] == V


def test_parareal_delta_and_stop(oracle):
    wl = W.ou_linear(P=300, N=5)
    pr = wl.problem
    u0 = oracle.sample_p0(pr, wl.P)
    res = oracle.parareal(pr, u0, 5, tol=1e9)
    assert res["iterations"] == 1  # delta <= tol stops after one iteration
    res = oracle.parareal(pr, u0, 5)
    d = res["delta"]
    # the last iterations only touch slices that are already exact or nearly
    assert d[-1] <= d[0]


# --------------------------------------------------------------------------- learning
def test_fraction_fit_recovers_exponential(oracle):
    """Two-region rate model dP1/dt = -w12 P1 + w21 P2: exact-exponential data
    P1(t) = P* + (P1(0) - P*) exp(-kappa t) is recovered."""
    kappa, pstar = 0.37, 0.62
    t = np.linspace(0, 4, 9)
    y = pstar + (0.5 - pstar) * np.exp(-kappa * t)
    k, p = oracle.fraction_fit(t, y, 0.1, y[-1])
    assert abs(k - kappa) < 1e-9 and abs(p - pstar) < 1e-9
    # conservation: the two fractions of the model sum to one
    w21 = kappa * pstar
    w12 = kappa - w21
    A = np.array([[-w12, w21], [w12, -w21]])
    assert np.allclose(A.sum(axis=0), 0.0)


def _relaxing_bimodal(P=1500, N=8, T=4.0):
    """Two-region double well whose particle fractions relax: an uneven
    mixture (95 % in the left well) with strong noise, so particles cross the
    barrier and the left fraction falls from 0.95 to about 0.73 over the horizon."""
    c = W.dz_coef(sigma=0.9)
    pr = W.make_problem(c, W.P0(W.P0_MIXTURE, 0.95, -1.0, 0.1, 1.0, 0.1), T, N, 1e-2, (0.0,))
    pr.coarse_model = W.COARSE_GAUSS3
    return W.Workload("relaxing_bimodal", pr, P, max_iter=N, learning=True)


def test_parareal_learning_keeps_exactness(oracle):
    """Learning-based MC-moments Parareal (Sec. 3.6): the extrapolated
    fractions touch only slices beyond the exact ones, so the exactness
    property still holds bit for bit and every exact slice takes the
    I(a, b, a) branch; and learning does change the slices beyond."""
    wl = _relaxing_bimodal()
    res, st = _invariant_check(oracle, wl, wl.problem.n_slices, learning=True)
    fl = res["flags"]
    for k in range(fl.shape[0]):
        assert np.all(fl[k, :k + 1] == 0), k
    fr = st[:, 0]["n"] / wl.P
    assert fr[0] - fr[-1] > 0.15  # the fractions do relax
    u0 = oracle.sample_p0(wl.problem, wl.P)
    plain = oracle.parareal(wl.problem, u0, 3)
    assert not np.array_equal(plain["rho"][2, :, :, 0], res["rho"][2, :, :, 0])


def test_parareal_learning_extrapolates_an_independent_fit(oracle):
    """After the fine sweep of iteration k the slices 0..k+1 are exact; their
    left-region fractions are fitted by the two-region rate model of App. H,
    P_1(t) = P* + (P_1(0) - P*) exp(-kappa t), and every later slice n of
    rho^{k+1} carries P* + (P_{1,k+1} - P*) exp(-kappa (t_n - t_{k+1})) in region
    0 and its complement in region 1.  The fit here is scipy's bounded
    trust-region least squares on the serial solution's fractions, a fitter
    and a data path that share nothing with the oracle's driver."""
    from scipy.optimize import least_squares
    wl = _relaxing_bimodal()
    pr, P, N = wl.problem, wl.P, wl.problem.n_slices
    u0 = oracle.sample_p0(pr, P)
    _, st = oracle.serial(pr, u0)
    y = st[:, 0]["n"] / P
    t = np.arange(N + 1) * pr.slice_length
    res = oracle.parareal(pr, u0, N, learning=True)
    checked = 0
    for k in range(1, res["iterations"]):
        tt, yy = t[:k + 2], y[:k + 2]
        fit = least_squares(lambda q: q[1] + (yy[0] - q[1]) * np.exp(-q[0] * tt) - yy,
                            x0=[1.0, 0.5], bounds=([0.0, 0.0], [np.inf, 1.0]),
                            xtol=1e-15, ftol=1e-15, gtol=1e-15, method="trf")
        kappa, pstar = fit.x
        for n in range(k + 2, N + 1):
            if res["flags"][k, n - 1, 0] == 0:
                continue  # (an I(a, b, a) short cut keeps the fine fractions)
            want = pstar + (yy[-1] - pstar) * math.exp(-kappa * (t[n] - t[k + 1]))
            rho = res["rho"][k + 1, n]
            assert abs(rho[0, 0] - want) <= 1e-8, (k, n, rho[0, 0], want)
            assert rho[1, 0] == 1.0 - rho[0, 0], (k, n)
            checked += 1
    assert checked >= 10


def test_parareal_learning_one_region_is_plain(oracle):
    """The fraction model needs two regions: with one region learning is a
    no-op, bit for bit."""
    wl = W.ou_linear(P=400, N=5)
    pr = wl.problem
    u0 = oracle.sample_p0(pr, wl.P)
    a = oracle.parareal(pr, u0, 4, keep_states=True)
    b = oracle.parareal(pr, u0, 4, keep_states=True, learning=True)
    for key in ("rho", "glob", "flags", "delta", "states"):
        np.testing.assert_array_equal(a[key], b[key])


@pytest.mark.parametrize("model,npts", [(W.COARSE_GAUSS2, 2), (W.COARSE_GAUSS3, 3)])
def test_gaussian_trig_field_hermite_nodes(oracle, model, npts):
    """Gaussian models of the plane rotator with two regions of positive
    variance: every expectation over N(M_i, V_i) -- the drift's own sin x term,
    the mean field's S = sum_i f_i E_i[sin X] and C = sum_i f_i E_i[cos X], and
    the moment equations' E[a], E[(x - M) a], E[b^2] -- taken with numpy's
    probabilists' Gauss-Hermite rule of the same order; the oracle's RK4
    against a tight solve of that system."""
    from numpy.polynomial.hermite_e import hermegauss
    K, kT = 1.2, 0.3
    pr = W.rotator(K=K, kT=kT, N=1, T=0.2).problem
    pr.splits = (math.pi,)
    pr.coarse_model = model
    pr.coarse_substeps = 40
    z, wz = hermegauss(npts)
    wz = wz / wz.sum()
    f = np.array([0.4, 0.6])
    y0 = np.array([1.0, 0.25, 4.0, 0.4])
    b = math.sqrt(2 * kT)

    def rhs(t, u):
        M, V = u[0::2], u[1::2]
        xs = [M[i] + np.sqrt(V[i]) * z for i in range(2)]
        S = sum(f[i] * wz @ np.sin(xs[i]) for i in range(2))
        C = sum(f[i] * wz @ np.cos(xs[i]) for i in range(2))
        out = []
        for i in range(2):
            a = -np.sin(xs[i]) + K * (S * np.cos(xs[i]) - C * np.sin(xs[i]))
            out += [wz @ a, 2 * wz @ ((xs[i] - M[i]) * a) + b * b]
        return out
    sol = solve_ivp(rhs, (0, pr.slice_length), y0, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(oracle.coarse(pr, f, y0), sol.y[:, -1], rtol=1e-9, atol=1e-12)
    # the rule matters: the point-mass field (the Taylor model's) is far off
    pr.coarse_model = W.COARSE_TAYLOR
    assert np.max(np.abs(oracle.coarse(pr, f, y0) - sol.y[:, -1])) > 1e-3


# --------------------------------------------------------------------------- classical Parareal
def test_classical_parareal_dahlquist(oracle):
    """A one-particle ensemble without noise is classical Parareal on the
    Dahlquist equation x' = lambda x (Sec. 4.2: R and M are the identity for a
    single particle): the fine propagator is explicit Euler, F = (1 + lambda
    dt)^m, the coarse one RK4, G = R(lambda h)^s with the RK4 stability
    polynomial.  Every iterate equals the textbook recursion
    U^{k+1}_{n+1} = G U^{k+1}_n + F U^k_n - G U^k_n, and at k = N the fine
    solution F^n U_0 is reached (Sec. 4.4)."""
    lam = -4.0
    N = 8
    pr = W.make_problem(W.Coef(a1=lam), W.P0(W.P0_DELTA, 1.0, 1.3, 0.0), 2.0, N, 0.05, coarse_h=0.25)
    assert pr.steps_per_slice == 5 and pr.coarse_substeps == 1
    m, s = pr.steps_per_slice, pr.coarse_substeps
    F = (1.0 + lam * pr.dt) ** m
    h = pr.slice_length / s
    z = lam * h
    G = (1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24) ** s
    u0 = oracle.sample_p0(pr, 1)
    assert u0[0] == 1.3
    res = oracle.parareal(pr, u0, N)
    assert res["iterations"] == N
    U = np.array([1.3 * G ** n for n in range(N + 1)])  # iteration 0: the coarse sweep
    fine = np.array([1.3 * F ** n for n in range(N + 1)])
    for k in range(N + 1):
        np.testing.assert_allclose(res["glob"][k, :, 0], U, rtol=1e-12, atol=0)
        assert np.all(res["glob"][k, :, 1] == 0.0)
        if k < N:
            Un = U.copy()
            for n in range(N):
                Un[n + 1] = G * Un[n] + F * U[n] - G * U[n]
            U = Un
    np.testing.assert_allclose(res["glob"][N, :, 0], fine, rtol=1e-12)
    # before k = N the coarse error is still visible at the last slice
    assert abs(res["glob"][N // 2, N, 0] - fine[N]) > 1e-3 * abs(fine[N])


def test_noisy_parareal_error_recursion_and_bounds(oracle):
    """MC-moments Parareal on the linear mean-field OU with the exact (Taylor)
    moment model: its mean is noisy classical Parareal (Lemma on the error
    recursion with noise).  The fine propagator maps slice means as
    M -> F M + f + eps_n, with eps_n the slice's statistical error (the
    per-realisation identity of the Euler-Maruyama mean), the coarse one as
    M -> G M + g.  Against the noise-free fine solution u_n (eps = 0) the mean
    iterates follow U^{k+1}_{n+1} = G U^{k+1}_n + g + F U^k_n + f + eps_n -
    (G U^k_n + g), and their error obeys the superlinear and the linear bound
    of the Lemma on Parareal with noise, with eps = max_n |eps_n|."""
    wl = W.ou_linear(P=2000, N=10, T=2.0)
    pr, P, N = wl.problem, wl.P, wl.problem.n_slices
    c = pr.coef
    lam, dt, m = c.a1 + c.am, pr.dt, pr.steps_per_slice
    F = (1.0 + lam * dt) ** m
    f = c.a0 * dt * sum((1.0 + lam * dt) ** j for j in range(m))
    h = pr.slice_length / pr.coarse_substeps
    z = lam * h
    R = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    G = R ** pr.coarse_substeps
    g = 0.0  # (a0 = 0)
    assert c.a0 == 0.0
    u0 = oracle.sample_p0(pr, P)
    _, st = oracle.serial(pr, u0)
    ms = np.array([s["mean"] for s in st[:, -1]])
    eps = ms[1:] - (F * ms[:-1] + f)
    res = oracle.parareal(pr, u0, N)
    assert np.all(res["flags"] <= 1)  # every region matched or short cut
    u = np.array([ms[0] * F ** n for n in range(N + 1)])  # noise-free fine solution (f = 0)
    U = res["glob"][0, :, 0].copy()
    xi0 = np.max(np.abs(U - u))
    E = np.max(np.abs(eps))
    for k in range(res["iterations"] + 1):
        got = res["glob"][k, :, 0]
        np.testing.assert_allclose(got, U, rtol=1e-11, atol=1e-13)
        xi = np.max(np.abs(got - u))
        sup = (abs(F - G) ** k / math.factorial(k) * math.prod(N - j for j in range(1, k + 1)) * xi0
               + E * (1 - abs(G) ** N) / (1 - abs(G)) * sum(abs(F - G) ** j * math.comb(N - 1, j)
                                                         for j in range(k)))
        q = abs(F - G) / (1 - abs(G))
        lin = q ** k * xi0 + E / (1 - abs(G)) * sum(q ** j for j in range(k))
        assert xi <= sup * (1 + 1e-9) + 1e-14, (k, xi, sup)
        assert xi <= lin * (1 + 1e-9) + 1e-14, (k, xi, lin)
        Un = U.copy()
        for n in range(N):
            Un[n + 1] = (G * Un[n] + g) + (F * U[n] + f + eps[n]) - (G * U[n] + g)
        U = Un


# --------------------------------------------------------------------------- adjoint
def _adjoint_problem(kind):
    """Both workload families, with every coefficient switched on (variance
    coupling and multiplicative noise included) so that each adjoint term is
    exercised."""
    if kind == "ou":
        c = W.Coef(a0=0.05, a1=-1.0, am=0.5, av=0.3, b0=0.3, b1=0.05, bm=0.05, bv=0.2)
        return W.make_problem(c, W.P0(W.P0_NORMAL, 1, 1.0, 0.2), 0.2, 4, 1e-2)
    c = W.dz_coef()
    c.av, c.bv, c.a2, c.b1 = 0.2, 0.1, 0.05, 0.02
    return W.make_problem(c, W.P0(W.P0_MIXTURE, 0.5, -1.0, 0.1, 1.0, 0.1), 0.2, 4, 1e-2, (0.0,))


@pytest.mark.parametrize("kind", ["ou", "dz"])
def test_adjoint_zero_at_targets_and_fd(oracle, kind):
    """Targets equal to the forward moments give J = 0 and a zero gradient;
    perturbed targets: the gradient matches central differences with common
    random numbers."""
    pr = _adjoint_problem(kind)
    P = 64
    x0 = oracle.sample_p0(pr, P)
    _, st = oracle.serial(pr, x0)
    Mh = np.array([s["mean"] for s in st[1:, -1]])
    Vh = np.array([s["var"] for s in st[1:, -1]])
    J, g = oracle.adjoint(pr, x0, Mh, Vh)
    assert J < 1e-28 and np.max(np.abs(g)) < 1e-12
    Mh2, Vh2 = Mh * 1.05 + 0.01, Vh * 0.9
    J, g = oracle.adjoint(pr, x0, Mh2, Vh2)
    names = ["a0", "a1", "a2", "a3", "am", "av", "b0", "b1", "bm", "bv"]
    for i, name in enumerate(names):
        h = 1e-6
        cp = W.Coef(**{**pr.coef.__dict__}); setattr(cp, name, getattr(cp, name) + h)
        cm = W.Coef(**{**pr.coef.__dict__}); setattr(cm, name, getattr(cm, name) - h)
        Jp, _ = oracle.adjoint(pr, x0, Mh2, Vh2, coef=cp)
        Jm, _ = oracle.adjoint(pr, x0, Mh2, Vh2, coef=cm)
        fd = (Jp - Jm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (name, fd, g[i])
