"""Seeded synthetic workloads: problem parameters and input recipes only.

This module holds no arithmetic of the method.  It describes each workload
(drift and diffusion coefficients, initial law, time grid, particle count,
regions, seed, precision) as plain data, and it is the one module that both
the HIP path and the CPU oracle are fed from.  Random numbers the method draws
are produced inside each implementation from the shared counter-based
convention (Philox4x32-10, counter = (particle quad, step, instance, tag));
the only draws made here are the per-instance parameters of the batched
workload, taken from numpy's seeded PCG64 generator.

The workloads stand in for the paper's experiments (Sec. 5): the linear
mean-field Ornstein-Uhlenbeck case (exact moment model, Lemma on exactness of
the Taylor model), the bimodal double-well case of Sec. 5.3 in its
Desai-Zwanzig mean-field form, a batch of independent OU instances, and the
large bimodal case with the particle-fraction learning of Sec. 3.6.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

FP64 = 0
FP32 = 1  # particle state in fp32, every reduction and the matching in fp64

COARSE_TAYLOR = 0
COARSE_GAUSS2 = 1
COARSE_GAUSS3 = 2

P0_NORMAL = 0
P0_MIXTURE = 1
P0_DELTA = 2


@dataclasses.dataclass
class Coef:
    """a(x,m,v) = a0 + a1 x + a2 x^2 + a3 x^3 + am m + av v + axs x (v + m^2);
    b(x,m,v) = b0 + b1 x + bm m + bv v."""
    a0: float = 0.0
    a1: float = 0.0
    a2: float = 0.0
    a3: float = 0.0
    am: float = 0.0
    av: float = 0.0
    b0: float = 0.0
    b1: float = 0.0
    bm: float = 0.0
    bv: float = 0.0
    axs: float = 0.0  # coefficient of x E[X^2]
    ksin: float = 0.0  # coefficient of sin x
    kc: float = 0.0  # coupling K of the mean field (1/P) sum_q sin(X_q - x)
    acdf: float = 0.0  # coefficient of 1 - F_P(x), F_P the empirical CDF with H(0) = 1/2

    def as_list(self) -> List[float]:
        return [self.a0, self.a1, self.a2, self.a3, self.am, self.av,
                self.b0, self.b1, self.bm, self.bv]


@dataclasses.dataclass
class P0:
    kind: int = P0_NORMAL
    w: float = 1.0
    mu1: float = 0.0
    sd1: float = 1.0
    mu2: float = 0.0
    sd2: float = 1.0


@dataclasses.dataclass
class Problem:
    coef: Coef
    p0: P0
    dt: float
    steps_per_slice: int
    n_slices: int
    splits: Sequence[float] = ()
    seed: int = 0
    coarse_substeps: int = 1
    precision: int = FP64
    coarse_model: int = 0  # 0 Taylor (eq. moment_model_class_1), 1/2 Gaussian with 2/3 sigma points
    wrap: int = 0  # 1: particles shifted modulo 2 pi into [0, 2 pi) after every step

    @property
    def n_regions(self) -> int:
        return len(self.splits) + 1

    @property
    def slice_length(self) -> float:
        return self.dt * self.steps_per_slice


@dataclasses.dataclass
class Workload:
    name: str
    problem: Problem
    P: int
    instances: List[dict] = dataclasses.field(default_factory=list)  # batched: [{P, coef, instance}]
    max_iter: int = 10
    tol: float = 0.0
    learning: bool = False


def steps_for(slice_length: float, dt_nominal: float) -> int:
    """Steps per slice: the slice length over the nominal step, rounded up
    unless it is an integer up to rounding."""
    r = slice_length / dt_nominal
    rr = round(r)
    if abs(r - rr) <= 1e-9 * max(1.0, r):
        return int(rr)
    return int(math.ceil(r))


def make_problem(coef: Coef, p0: P0, T: float, N: int, dt_nominal: float, splits=(),
                 seed: int = 0, coarse_h: float = 0.05, precision: int = FP64) -> Problem:
    dT = T / N
    m = steps_for(dT, dt_nominal)
    dt = dT / m
    sub = steps_for(dT, coarse_h) if dT > coarse_h else 1
    return Problem(coef=coef, p0=p0, dt=dt, steps_per_slice=m, n_slices=N, splits=tuple(splits),
                   seed=seed, coarse_substeps=max(1, sub), precision=precision)


# --- the workload family -------------------------------------------------------

def ou_coef(theta: float = 1.0, sigma: float = 0.3, am: float = 0.5) -> Coef:
    """Linear mean-field OU: dX = (-theta X + am E[X]) dt + sigma dW."""
    return Coef(a1=-theta, am=am, b0=sigma)


def dz_coef(sigma: float = 0.5) -> Coef:
    """Desai-Zwanzig double well with mean-field attraction:
    dX = (X - X^3 - 0.5 (X - E[X])) dt + sigma dW."""
    return Coef(a1=0.5, a3=-1.0, am=0.5, b0=sigma)


def ou_linear(P: int = 10_000, precision: int = FP64, N: int = 10, T: float = 1.0,
              dt: float = 1e-3, seed: int = 0) -> Workload:
    """Linear mean-field OU, X0 ~ N(1, 0.2^2), P = 1e4, T = 1, dt = 1e-3, N = 10,
    RK4 coarse step 0.05, fp64, up to 10 iterations."""
    pr = make_problem(ou_coef(), P0(P0_NORMAL, 1.0, 1.0, 0.2), T, N, dt, (), seed, 0.05, precision)
    return Workload("ou_linear", pr, P, max_iter=N, tol=0.0)


def gbm_coef() -> Coef:
    """Geometric Brownian motion with interaction (the nonlinear-QoI example of
    Sec. 5.1): dX = (alpha X + beta E[X] + a) dt + (sigma X + omega E[X] + b) dW,
    alpha = -1/2, beta = 4/5, a = 1/3, sigma = omega = (1/2) sqrt(1/2), b = 1/6."""
    s = 0.5 * math.sqrt(0.5)
    return Coef(a0=1.0 / 3.0, a1=-0.5, am=0.8, b0=1.0 / 6.0, b1=s, bm=s)


def gbm(P: int = 100_000, precision: int = FP64, N: int = 10, T: float = 1.0, dt: float = 1e-3,
        seed: int = 0, coarse_model: int = 0) -> Workload:
    """Geometric Brownian motion with interaction and the QoI sin(x^2):
    X0 ~ N(1, 1/4) (variance 1/4: standard deviation 1/2), one region; the
    paper prints no horizon or sizes, so T = 1, N = 10, dt = 1e-3, P = 1e5."""
    pr = make_problem(gbm_coef(), P0(P0_NORMAL, 1.0, 1.0, 0.5), T, N, dt, (), seed, 0.05, precision)
    pr.coarse_model = coarse_model
    return Workload("gbm", pr, P, max_iter=N, tol=0.0)


def polydrift(P: int = 100_000, precision: int = FP64, N: int = 10, T: float = 2.0, dt: float = 1e-3,
              alpha: float = 0.5, seed: int = 0, coarse_model: int = 0) -> Workload:
    """Polynomial drift dX = (alpha X + E[X] - X E[X^2]) dt + X dW, X(0) = 1
    (the example of the appendix on the exactness of the moment model; the
    Taylor model is its exact moment system).  alpha is not printed there:
    alpha = 1/2, for which (M, E[X^2]) settle at (sqrt(3)/2, 3/2)."""
    pr = make_problem(Coef(a1=alpha, am=1.0, axs=-1.0, b1=1.0), P0(P0_DELTA, 1.0, 1.0, 0.0), T, N, dt, (),
                      seed, 0.05, precision)
    pr.coarse_model = coarse_model
    return Workload("polydrift", pr, P, max_iter=N, tol=0.0)


def rotator(P: int = 100_000, precision: int = FP64, N: int = 20, T: float = 10.0, dt: float = 1e-3,
            K: float = 1.0, kT: float = 0.5, wrap: int = 1, seed: int = 0, coarse_model: int = 0) -> Workload:
    """Plane rotator (Sec. 5.1): dX = [K E_q[sin(X_q - X)] - sin X] dt + sqrt(2 kB T) dW,
    X0 ~ N(pi/4, 3 pi/4) (variance 3 pi/4), shifted modulo 2 pi into [0, 2 pi)
    after every step; T = 10, dt = 1e-3, 1e5 particles as in the paper.  K and
    kB T are not printed: K = 1, kB T = 1/2 (unit noise)."""
    pr = make_problem(Coef(ksin=-1.0, kc=K, b0=math.sqrt(2.0 * kT)),
                      P0(P0_NORMAL, 1.0, math.pi / 4, math.sqrt(3 * math.pi / 4)), T, N, dt, (), seed, 0.05,
                      precision)
    pr.coarse_model = coarse_model
    pr.wrap = wrap
    return Workload("rotator", pr, P, max_iter=N, tol=0.0)


def burgers(P: int = 100_000, precision: int = FP64, N: int = 10, T: float = 1.0, dt: float = 1e-3,
            sigma: float = 1.0, seed: int = 0) -> Workload:
    """Particle system of the viscous Burgers equation (Sec. 5.2):
    dX = (1 - F_P(X)) dt + sigma dW, X(0) = 0, F_P the empirical CDF with
    H(0) = 1/2; the coarse propagator is the Gaussian-density moment model
    dM = 1/2, dSigma = -(2 / sqrt(2 pi)) sqrt(Sigma) + sigma^2.  sigma and the
    horizon are not printed: sigma = 1, T = 1, N = 10."""
    pr = make_problem(Coef(acdf=1.0, b0=sigma), P0(P0_DELTA, 1.0, 0.0, 0.0), T, N, dt, (), seed, 0.05, precision)
    return Workload("burgers", pr, P, max_iter=N, tol=0.0)


def dz_bimodal(P: int = 1_000_000, precision: int = FP32, N: int = 50, T: float = 5.0,
               dt: float = 1e-3, seed: int = 0) -> Workload:
    """Bimodal Desai-Zwanzig, X0 ~ 0.5 N(-1, 0.1^2) + 0.5 N(1, 0.1^2), P = 1e6,
    T = 5, dt = 1e-3, N = 50, two regions split at 0, fp32 state / fp64 reductions."""
    pr = make_problem(dz_coef(), P0(P0_MIXTURE, 0.5, -1.0, 0.1, 1.0, 0.1), T, N, dt, (0.0,), seed,
                      0.05, precision)
    return Workload("dz_bimodal", pr, P, max_iter=N, tol=0.0)


def ou_batched(n_inst: int = 64, N: int = 32, T: float = 1.0, dt: float = 1e-3,
               p_lo: float = 1e4, p_hi: float = 2e6, seed: int = 0,
               precision: int = FP32) -> Workload:
    """64 independent OU instances, theta ~ U[0.1, 1], sigma ~ U[0.2, 0.8],
    P log-uniform in [1e4, 2e6], N = 32 slices each, T = 1 (dt_eff = 1/1024)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = rng.uniform(0.1, 1.0, n_inst)
    sigma = rng.uniform(0.2, 0.8, n_inst)
    P = np.rint(np.exp(rng.uniform(math.log(p_lo), math.log(p_hi), n_inst))).astype(np.int64)
    pr = make_problem(ou_coef(), P0(P0_NORMAL, 1.0, 1.0, 0.2), T, N, dt, (), seed, 0.05, precision)
    inst = [dict(P=int(P[i]), coef=ou_coef(float(theta[i]), float(sigma[i])), instance=i)
            for i in range(n_inst)]
    return Workload("ou_batched", pr, int(P.sum()), instances=inst, max_iter=N)


def adjoint_case(kind: str = "ou", P: int = 100_000, precision: int = FP32) -> Workload:
    """Adjoint workload: T = 2, dt = 1e-3, N = 20 (checkpoint every 100 steps)."""
    if kind == "ou":
        pr = make_problem(ou_coef(), P0(P0_NORMAL, 1.0, 1.0, 0.2), 2.0, 20, 1e-3, (), 0, 0.05, precision)
    else:
        pr = make_problem(dz_coef(), P0(P0_MIXTURE, 0.5, -1.0, 0.1, 1.0, 0.1), 2.0, 20, 1e-3, (0.0,),
                          0, 0.05, precision)
    return Workload("adjoint_" + kind, pr, P)


def dz_large(P: int = 16_000_000, N: int = 256, T: float = 10.0, dt: float = 5e-4,
             tol: float = 1e-4, seed: int = 0) -> Workload:
    """Large bimodal DZ with the fraction-learning extension: P = 1.6e7, N = 256,
    T = 10, dt = 5e-4 (79 steps per slice), fp32 state, tolerance 1e-4.  The
    coarse propagator is the Gaussian model with three sigma points: the
    second-order Taylor model has no equilibrium for this drift and its
    trajectory diverges before T = 10."""
    pr = make_problem(dz_coef(), P0(P0_MIXTURE, 0.5, -1.0, 0.1, 1.0, 0.1), T, N, dt, (0.0,), seed,
                      0.05, FP32)
    pr.coarse_model = COARSE_GAUSS3
    return Workload("dz_large", pr, P, max_iter=N, tol=tol, learning=True)
