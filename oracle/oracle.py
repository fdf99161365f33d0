"""ctypes binding of the FP64 CPU oracle (oracle/mcpr_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and by
the cpu_baseline leg of bench.py.  The product path never imports it.  It
shares no code with the HIP library; both are fed the same plain-data problem
description (paper_2310_11365_amd.workloads.Problem, duck-typed here).

Each wrapper names the passage of the paper its C function follows; see the
header of mcpr_oracle.c.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "mcpr_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")

BUILD_CMD = ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", LIB, SRC, "-lm"]


def build(force: bool = True) -> str:
    """Compile the oracle (plain C, FP64, no FMA contraction)."""
    if force or not os.path.exists(LIB):
        subprocess.check_call(BUILD_CMD)
    return LIB


class OrProblem(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("a0", "a1", "a2", "a3", "am", "av", "b0", "b1", "bm", "bv", "axs",
                                               "ksin", "kc", "acdf")] + [
        ("p0_kind", ctypes.c_int32), ("pad0", ctypes.c_int32),
        ("p0_w", ctypes.c_double), ("p0_mu1", ctypes.c_double), ("p0_sd1", ctypes.c_double),
        ("p0_mu2", ctypes.c_double), ("p0_sd2", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("steps_per_slice", ctypes.c_int32), ("n_slices", ctypes.c_int32),
        ("n_regions", ctypes.c_int32), ("coarse_substeps", ctypes.c_int32),
        ("split", ctypes.c_double * 7),
        ("seed", ctypes.c_uint64),
        ("coarse_model", ctypes.c_int32), ("wrap", ctypes.c_int32),
    ]


class OrStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("mean", ctypes.c_double), ("var", ctypes.c_double),
                ("min", ctypes.c_double), ("max", ctypes.c_double)]


STATS_DTYPE = np.dtype([("n", np.int64), ("mean", np.float64), ("var", np.float64),
                        ("min", np.float64), ("max", np.float64)])

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        pp = ctypes.POINTER(OrProblem)
        sp = ctypes.c_void_p
        L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.or_uniform.argtypes = [ctypes.c_uint32]
        L.or_uniform.restype = ctypes.c_double
        L.or_normals4.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.c_uint32, dp]
        L.or_sample_p0.argtypes = [pp, ctypes.c_int64, ctypes.c_uint32, dp]
        L.or_moments.argtypes = [dp, ctypes.c_int64, dp, dp]
        L.or_region_of.argtypes = [pp, ctypes.c_double]
        L.or_region_of.restype = ctypes.c_int
        L.or_restrict.argtypes = [pp, dp, ctypes.c_int64, sp]
        L.or_fine.argtypes = [pp, dp, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32, dp]
        L.or_coarse.argtypes = [pp, dp, dp, dp]
        L.or_transform.argtypes = [pp, dp, dp, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32,
                                   ctypes.c_int, sp, ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.or_transform.restype = ctypes.c_int
        L.or_rho_global.argtypes = [ctypes.c_int, dp, dp, dp]
        L.or_fraction_fit.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_double, dp, dp]
        L.or_serial.argtypes = [pp, dp, ctypes.c_int64, ctypes.c_uint32, sp]
        L.or_empirical_cdf.argtypes = [dp, ctypes.c_int64, dp]
        L.or_empirical_cdf.restype = None
        L.or_qoi.argtypes = [dp, ctypes.c_int64, ctypes.c_int32]
        L.or_qoi.restype = ctypes.c_double
        L.or_parareal.argtypes = [pp, dp, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_double,
                                  ctypes.c_int32, dp, dp, dp, ctypes.POINTER(ctypes.c_int32), dp, dp]
        L.or_parareal.restype = ctypes.c_int
        L.or_adjoint.argtypes = [pp, dp, ctypes.c_int64, ctypes.c_uint32, dp, dp, dp]
        L.or_adjoint.restype = ctypes.c_double
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def to_c(problem, coef=None) -> OrProblem:
    """Convert a workloads.Problem (optionally with an instance's coefficients)."""
    c = coef if coef is not None else problem.coef
    s = OrProblem()
    for name in ("a0", "a1", "a2", "a3", "am", "av", "b0", "b1", "bm", "bv", "axs", "ksin", "kc", "acdf"):
        setattr(s, name, float(getattr(c, name, 0.0)))
    s.p0_kind = int(problem.p0.kind)
    s.p0_w, s.p0_mu1, s.p0_sd1 = float(problem.p0.w), float(problem.p0.mu1), float(problem.p0.sd1)
    s.p0_mu2, s.p0_sd2 = float(problem.p0.mu2), float(problem.p0.sd2)
    s.dt = float(problem.dt)
    s.steps_per_slice = int(problem.steps_per_slice)
    s.n_slices = int(problem.n_slices)
    s.n_regions = int(problem.n_regions)
    s.coarse_substeps = int(problem.coarse_substeps)
    for i, v in enumerate(problem.splits):
        s.split[i] = float(v)
    s.seed = int(problem.seed)
    s.coarse_model = int(getattr(problem, "coarse_model", 0))
    s.wrap = int(getattr(problem, "wrap", 0))
    return s


# ---------------------------------------------------------------------------
def philox(ctr, key):
    """Philox4x32-10 block function on one 128-bit counter and 64-bit key."""
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def uniform(w: int) -> float:
    return lib().or_uniform(w)


def normals4(seed, q, s, inst, tag) -> np.ndarray:
    z = np.zeros(4)
    lib().or_normals4(seed, q, s, inst, tag, _dp(z))
    return z


def sample_p0(problem, P, inst=0, coef=None) -> np.ndarray:
    x = np.zeros(P)
    pr = to_c(problem, coef)
    lib().or_sample_p0(ctypes.byref(pr), P, inst, _dp(x))
    return x


def moments(x: np.ndarray):
    x = np.ascontiguousarray(x, dtype=np.float64)
    m, v = ctypes.c_double(), ctypes.c_double()
    lib().or_moments(_dp(x), x.size, ctypes.byref(m), ctypes.byref(v))
    return m.value, v.value


QOI_X, QOI_X2, QOI_SIN_X2 = 0, 1, 2


def qoi(x: np.ndarray, kind: int) -> float:
    """(1/P) sum Phi(x_p); kind 0: x, 1: x^2, 2: sin(x^2)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(lib().or_qoi(_dp(x), x.size, kind))


def empirical_cdf(x: np.ndarray) -> np.ndarray:
    """F[p] = (1/P) sum_q H(x_p - x_q), H(0) = 1/2."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    F = np.zeros_like(x)
    lib().or_empirical_cdf(_dp(x), x.size, _dp(F))
    return F


def region_of(problem, x: float) -> int:
    pr = to_c(problem)
    return lib().or_region_of(ctypes.byref(pr), float(x))


def restrict(problem, x: np.ndarray) -> np.ndarray:
    """Per-region (n, mean, var, min, max); the last entry is the whole ensemble."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(problem.n_regions + 1, dtype=STATS_DTYPE)
    pr = to_c(problem)
    lib().or_restrict(ctypes.byref(pr), _dp(x), x.size, out.ctypes.data)
    return out


def fine(problem, x: np.ndarray, slice_index: int, inst=0, coef=None, trace=False):
    """F_n in place on a float64 copy; returns (x_new, trace[m,2] or None)."""
    x = np.array(x, dtype=np.float64, copy=True)
    pr = to_c(problem, coef)
    tr = np.zeros((problem.steps_per_slice, 2)) if trace else None
    lib().or_fine(ctypes.byref(pr), _dp(x), x.size, inst, slice_index,
                  _dp(tr) if trace else ctypes.POINTER(ctypes.c_double)())
    return x, tr


def coarse(problem, fractions, y, coef=None) -> np.ndarray:
    """One coarse slice: y = (M_1, V_1, ..., M_I, V_I), fractions frozen."""
    f = np.ascontiguousarray(fractions, dtype=np.float64)
    yi = np.ascontiguousarray(y, dtype=np.float64)
    yo = np.zeros_like(yi)
    pr = to_c(problem, coef)
    lib().or_coarse(ctypes.byref(pr), _dp(f), _dp(yi), _dp(yo))
    return yo


def transform(problem, x, region, src_stats, mu, sigma, boundary=0, inst=0, apply=True):
    """T([mu, sigma], u) on the particles of one region; returns (x_new, inside)."""
    xi = np.ascontiguousarray(x, dtype=np.float64)
    y = xi.copy()
    st = OrStats(int(src_stats["n"]), float(src_stats["mean"]), float(src_stats["var"]),
                 float(src_stats["min"]), float(src_stats["max"]))
    pr = to_c(problem)
    inside = lib().or_transform(ctypes.byref(pr), _dp(xi), _dp(y), xi.size, inst, boundary, region,
                                ctypes.byref(st), float(mu), float(sigma), 1 if apply else 0)
    return y, bool(inside)


def rho_global(rho: np.ndarray):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    M, V = ctypes.c_double(), ctypes.c_double()
    lib().or_rho_global(rho.size // 3, _dp(rho), ctypes.byref(M), ctypes.byref(V))
    return M.value, V.value


def fraction_fit(t, y, kappa0, pstar0):
    t = np.ascontiguousarray(t, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    k, p = ctypes.c_double(), ctypes.c_double()
    lib().or_fraction_fit(t.size, _dp(t), _dp(y), kappa0, pstar0, ctypes.byref(k), ctypes.byref(p))
    return k.value, p.value


def serial(problem, x0: np.ndarray, inst=0, coef=None):
    """Serial fine solution; returns (x_N, stats[(N+1), I+1])."""
    x = np.array(x0, dtype=np.float64, copy=True)
    st = np.zeros((problem.n_slices + 1, problem.n_regions + 1), dtype=STATS_DTYPE)
    pr = to_c(problem, coef)
    lib().or_serial(ctypes.byref(pr), _dp(x), x.size, inst, st.ctypes.data)
    return x, st


def parareal(problem, u0: np.ndarray, K: int, tol: float = 0.0, inst=0, learning=False,
             keep_states=False, coef=None, fractions=None):
    """MC-moments Parareal; returns a dict with rho[k,n,i,3], glob[k,n,2],
    flags[k,n,i], delta[k], iterations, and optionally states[k,n,P].
    fractions: optional [N+1, I] given particle fractions of every macro state."""
    N, I = problem.n_slices, problem.n_regions
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    P = u0.size
    rho = np.zeros((K + 1, N + 1, I, 3))
    glob = np.zeros((K + 1, N + 1, 2))
    flags = np.full((K, N, I), -1, dtype=np.int32)
    delta = np.zeros(max(K, 1))
    states = np.zeros((K + 1, N + 1, P)) if keep_states else None
    pr = to_c(problem, coef)
    fr = None
    if fractions is not None:
        fr = np.ascontiguousarray(fractions, dtype=np.float64).reshape(N + 1, I)
    null = ctypes.POINTER(ctypes.c_double)()
    its = lib().or_parareal(ctypes.byref(pr), _dp(u0), P, inst, K, tol, 1 if learning else 0,
                            _dp(fr) if fr is not None else null, _dp(rho), _dp(glob),
                            flags.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(delta),
                            _dp(states) if keep_states else null)
    out = dict(rho=rho[:its + 1], glob=glob[:its + 1], flags=flags[:its], delta=delta[:its], iterations=its)
    if keep_states:
        out["states"] = states[:its + 1]
    return out


def adjoint(problem, x0, Mhat, Vhat, inst=0, coef=None):
    """J and dJ/d(a0,a1,a2,a3,am,av,b0,b1,bm,bv) through the serial fine solution."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    Mh = np.ascontiguousarray(Mhat, dtype=np.float64)
    Vh = np.ascontiguousarray(Vhat, dtype=np.float64)
    g = np.zeros(10)
    pr = to_c(problem, coef)
    J = lib().or_adjoint(ctypes.byref(pr), _dp(x0), x0.size, inst, _dp(Mh), _dp(Vh), _dp(g))
    return J, g
