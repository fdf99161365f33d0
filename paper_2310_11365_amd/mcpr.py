"""ctypes binding of libmcpr.so (C ABI in include/mcpr.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  PyTorch provides device memory and streams.  If the library is
missing the binding raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcpr.so")

FP64, FP32 = 0, 1
MAP_KEEP, MAP_AFFINE, MAP_RESAMPLE = 0, 1, 2
QOI_X, QOI_X2, QOI_SIN_X2 = 0, 1, 2
MAX_REGIONS = 8

STATUS = {0: "MCPR_OK", -1: "MCPR_E_INVALID_ARG", -2: "MCPR_E_OOM", -3: "MCPR_E_DEVICE",
          -4: "MCPR_E_NONFINITE", -5: "MCPR_E_UNSUPPORTED", -6: "MCPR_E_NOT_RESERVED"}
RESERVE_INIT, RESERVE_MOMENTS, RESERVE_QOI, RESERVE_FINE, RESERVE_MATCH, RESERVE_ADJOINT = 1, 2, 4, 8, 16, 32


class MCPRError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Coef(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("a0", "a1", "a2", "a3", "am", "av", "b0", "b1", "bm", "bv", "axs",
                                               "ksin", "kc", "acdf")]


class ProblemC(ctypes.Structure):
    _fields_ = [("coef", Coef), ("p0_kind", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("p0_w", ctypes.c_double), ("p0_mu1", ctypes.c_double), ("p0_sd1", ctypes.c_double),
                ("p0_mu2", ctypes.c_double), ("p0_sd2", ctypes.c_double), ("dt", ctypes.c_double),
                ("steps_per_slice", ctypes.c_int32), ("n_slices", ctypes.c_int32),
                ("n_regions", ctypes.c_int32), ("coarse_substeps", ctypes.c_int32),
                ("split", ctypes.c_double * (MAX_REGIONS - 1)), ("seed", ctypes.c_uint64),
                ("coarse_model", ctypes.c_int32), ("wrap", ctypes.c_int32)]


class EnsembleC(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("n_particles", ctypes.c_int64), ("instance", ctypes.c_int32),
                ("slice", ctypes.c_int32), ("problem", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class InstanceC(ctypes.Structure):
    _fields_ = [("problem", ctypes.c_int32), ("instance", ctypes.c_int32), ("n_particles", ctypes.c_int64),
                ("slot_stride", ctypes.c_int64), ("ring", ctypes.c_void_p)]


STATS_DTYPE = np.dtype([("n", np.int64), ("mean", np.float64), ("var", np.float64), ("min", np.float64),
                        ("max", np.float64), ("nonfinite", np.int32), ("reserved", np.int32)])
MAP_DTYPE = np.dtype([("from", np.float64), ("scale", np.float64), ("to", np.float64), ("mode", np.int32),
                      ("boundary", np.int32)])
assert STATS_DTYPE.itemsize == 48 and MAP_DTYPE.itemsize == 32

_lib = None


def lib() -> ctypes.CDLL:
    """Load libmcpr.so (torch is imported first so that the process has one HIP runtime)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads the HIP runtime the library binds to)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int
        pP, pE = ctypes.POINTER(ProblemC), ctypes.POINTER(EnsembleC)
        L.mcpr_create.argtypes = [ctypes.POINTER(vp), i32]
        L.mcpr_create.restype = st
        L.mcpr_destroy.argtypes = [vp]
        L.mcpr_destroy.restype = None
        L.mcpr_last_error.argtypes = [vp]
        L.mcpr_last_error.restype = ctypes.c_char_p
        L.mcpr_version.restype = ctypes.c_char_p
        L.mcpr_reserve.argtypes = [vp, pP, i32, pE, i32, i32]
        L.mcpr_reserve.restype = st
        L.mcpr_alloc_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.mcpr_alloc_stats.restype = st
        L.mcpr_init_particles.argtypes = [vp, pP, i32, pE, i32, vp]
        L.mcpr_init_particles.restype = st
        L.mcpr_moments.argtypes = [vp, pP, i32, pE, i32, vp, vp]
        L.mcpr_moments.restype = st
        L.mcpr_qoi.argtypes = [vp, pP, i32, pE, i32, i32, vp, vp]
        L.mcpr_qoi.restype = st
        L.mcpr_fine_propagate.argtypes = [vp, pP, i32, pE, i32, vp, vp, vp]
        L.mcpr_fine_propagate.restype = st
        L.mcpr_fine_propagate_static.argtypes = [pP, i32, pE, i32, vp, vp, vp]
        L.mcpr_fine_propagate_static.restype = st
        L.mcpr_match.argtypes = [vp, pP, i32, pE, i32, vp, i32, vp, vp]
        L.mcpr_match.restype = st
        L.mcpr_profile_enable.argtypes = [vp, i32]
        L.mcpr_profile_enable.restype = st
        L.mcpr_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64), i32]
        L.mcpr_profile_read.restype = st
        L.mcpr_profile_read_adjoint.argtypes = L.mcpr_profile_read.argtypes
        L.mcpr_profile_read_adjoint.restype = st
        L.mcpr_stream_probe.argtypes = [vp, ctypes.c_int64, i32, vp, ctypes.POINTER(ctypes.c_double)]
        L.mcpr_stream_probe.restype = st
        L.mcpr_set_graphs.argtypes = [vp, i32]
        L.mcpr_set_graphs.restype = st
        L.mcpr_set_tuning.argtypes = [vp, i32]
        L.mcpr_set_tuning.restype = st
        L.mcpr_tuned_variant.argtypes = [vp, i32]
        L.mcpr_tuned_variant.restype = i32
        L.mcpr_graph_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.mcpr_graph_stats.restype = st
        L.mcpr_set_resident.argtypes = [vp, i32]
        L.mcpr_set_resident.restype = st
        L.mcpr_resident_sweeps.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.mcpr_resident_sweeps.restype = st
        L.mcpr_set_cdf_sort.argtypes = [vp, i32]
        L.mcpr_set_cdf_sort.restype = st
        L.mcpr_cdf_stats.argtypes = [vp] + [ctypes.POINTER(ctypes.c_int64)] * 3
        L.mcpr_cdf_stats.restype = st
        L.mcpr_adjoint.argtypes = [vp, pP, pE, vp, vp, vp, vp]
        L.mcpr_adjoint.restype = st
        L.mcpr_parareal_create.argtypes = [vp, pP, i32, ctypes.POINTER(InstanceC), i32, i32, ctypes.c_double,
                                           ctypes.POINTER(vp)]
        L.mcpr_parareal_create.restype = st
        L.mcpr_parareal_destroy.argtypes = [vp]
        L.mcpr_parareal_destroy.restype = None
        L.mcpr_parareal_init.argtypes = [vp, i32, vp]
        L.mcpr_parareal_init.restype = st
        L.mcpr_parareal_iterate.argtypes = [vp, ctypes.POINTER(ctypes.c_double), vp]
        L.mcpr_parareal_iterate.restype = st
        L.mcpr_parareal_iteration.argtypes = [vp]
        L.mcpr_parareal_iteration.restype = i32
        L.mcpr_parareal_qoi.argtypes = [vp, i32, i32, vp, vp]
        L.mcpr_parareal_qoi.restype = st
        L.mcpr_parareal_track_qoi.argtypes = [vp, i32]
        L.mcpr_parareal_track_qoi.restype = st
        L.mcpr_parareal_macro.argtypes = [vp, i32, vp, vp]
        L.mcpr_parareal_macro.restype = st
        L.mcpr_parareal_set_fractions.argtypes = [vp, i32, vp]
        L.mcpr_parareal_set_fractions.restype = st
        L.mcpr_parareal_flags.argtypes = [vp, i32, vp]
        L.mcpr_parareal_flags.restype = st
        L.mcpr_parareal_save.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
        L.mcpr_parareal_save.restype = st
        L.mcpr_parareal_restore.argtypes = [vp, vp, ctypes.c_size_t]
        L.mcpr_parareal_restore.restype = st
        L.mcpr_parareal_slot.argtypes = [vp, i32, i32, ctypes.POINTER(vp)]
        L.mcpr_parareal_slot.restype = st
        _lib = L
    return _lib


def problem_c(problem, coef=None) -> ProblemC:
    """workloads.Problem (plus optional per-instance coefficients) -> mcpr_problem."""
    c = coef if coef is not None else problem.coef
    s = ProblemC()
    for n in ("a0", "a1", "a2", "a3", "am", "av", "b0", "b1", "bm", "bv", "axs", "ksin", "kc", "acdf"):
        setattr(s.coef, n, float(getattr(c, n, 0.0)))
    s.p0_kind = int(problem.p0.kind)
    s.precision = int(problem.precision)
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


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _ptr(t) -> int:
    return t.data_ptr() if hasattr(t, "data_ptr") else int(t)


def torch_dtype(precision: int):
    import torch
    return torch.float64 if precision == FP64 else torch.float32


class Context:
    """A library context on one device (owns the reduction scratch)."""

    def __init__(self, device: int = 0):
        L = lib()
        h = ctypes.c_void_p()
        st = L.mcpr_create(ctypes.byref(h), int(device))
        if st != 0:
            raise MCPRError(st, "mcpr_create failed")
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            lib().mcpr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def _check(self, st: int):
        if st != 0:
            raise MCPRError(st, lib().mcpr_last_error(self._h).decode())

    @staticmethod
    def _arrays(problems, ensembles):
        P = (ProblemC * len(problems))(*problems)
        E = (EnsembleC * len(ensembles))(*ensembles)
        return P, E

    def profile(self, on: bool):
        self._check(lib().mcpr_profile_enable(self._h, 1 if on else 0))

    def profile_read(self, reset: bool = True):
        """(elapsed ms of the step launches, number of step launches, particle-steps)."""
        ms, n, ps = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().mcpr_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(ps),
                                            1 if reset else 0))
        return ms.value, n.value, ps.value

    def profile_read_adjoint(self, reset: bool = True):
        """(elapsed ms of the adjoint's backward step launches, backward steps, particle-steps)."""
        ms, n, ps = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().mcpr_profile_read_adjoint(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(ps),
                                                    1 if reset else 0))
        return ms.value, n.value, ps.value

    def set_graphs(self, on: bool):
        self._check(lib().mcpr_set_graphs(self._h, 1 if on else 0))

    def set_tuning(self, mode: int):
        """-1: autotune the step-kernel variant per launch shape; 0..3: force one
        (bit 0 non-temporal, bit 1 separate mean-field combine)."""
        self._check(lib().mcpr_set_tuning(self._h, int(mode)))

    def tuned_variants(self):
        out, i = [], 0
        while True:
            v = lib().mcpr_tuned_variant(self._h, i)
            if v < 0:
                return out
            out.append(v)
            i += 1

    def graph_stats(self):
        b, n = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().mcpr_graph_stats(self._h, ctypes.byref(b), ctypes.byref(n)))
        return b.value, n.value

    def set_resident(self, enable: bool):
        """Resident fine sweeps of small ensembles (default on; the same bits
        as the per-step launches)."""
        self._check(lib().mcpr_set_resident(self._h, 1 if enable else 0))

    def resident_sweeps(self) -> int:
        """Fine sweeps run resident so far."""
        v = ctypes.c_int64()
        self._check(lib().mcpr_resident_sweeps(self._h, ctypes.byref(v)))
        return v.value

    def set_cdf_sort(self, mode: int):
        """Sort of the empirical-CDF drift: 1 buckets after each sweep's first
        steps (default), 0 the radix sort on every step (both give the same
        bits)."""
        self._check(lib().mcpr_set_cdf_sort(self._h, int(mode)))

    def cdf_stats(self):
        """(bucket sweeps, radix-sort-only sweeps, sweeps redone after an overflow)."""
        v = [ctypes.c_int64() for _ in range(3)]
        self._check(lib().mcpr_cdf_stats(self._h, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def reserve(self, problems, ensembles, calls: int):
        """mcpr_reserve: size the context's scratch for later calls of the
        kinds in calls (RESERVE_*) on these ensembles (allocates only what is
        not held yet)."""
        P, E = self._arrays(problems, ensembles)
        self._check(lib().mcpr_reserve(self._h, P, len(problems), E, len(ensembles), int(calls)))

    def alloc_stats(self):
        """(allocations, bytes) the context and its drivers have made so far."""
        n, b = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().mcpr_alloc_stats(self._h, ctypes.byref(n), ctypes.byref(b)))
        return n.value, b.value

    # The methods below reserve before each call (a no-op once the scratch
    # suffices), so that Python callers need not size the context themselves.
    def init_particles(self, problems: Sequence[ProblemC], ensembles: Sequence[EnsembleC], stream=None):
        P, E = self._arrays(problems, ensembles)
        self._check(lib().mcpr_reserve(self._h, P, len(problems), E, len(ensembles), RESERVE_INIT))
        self._check(lib().mcpr_init_particles(self._h, P, len(problems), E, len(ensembles), _stream(stream)))

    def moments(self, problems, ensembles, stats_dev, stream=None):
        """stats_dev: a device tensor of >= n_ens*(I+1)*48 bytes."""
        P, E = self._arrays(problems, ensembles)
        self._check(lib().mcpr_reserve(self._h, P, len(problems), E, len(ensembles), RESERVE_MOMENTS))
        self._check(lib().mcpr_moments(self._h, P, len(problems), E, len(ensembles), _ptr(stats_dev),
                                       _stream(stream)))

    def qoi(self, problems, ensembles, kind: int, out_dev, stream=None):
        """out_dev: a float64 device tensor of >= n_ens entries; out[e] = (1/P) sum Phi(x)."""
        P, E = self._arrays(problems, ensembles)
        self._check(lib().mcpr_reserve(self._h, P, len(problems), E, len(ensembles), RESERVE_QOI))
        self._check(lib().mcpr_qoi(self._h, P, len(problems), E, len(ensembles), int(kind), _ptr(out_dev),
                                   _stream(stream)))

    def fine_propagate(self, problems, ensembles, stats_dev=None, trace_dev=None, stream=None):
        P, E = self._arrays(problems, ensembles)
        self._check(lib().mcpr_reserve(self._h, P, len(problems), E, len(ensembles), RESERVE_FINE))
        self._check(lib().mcpr_fine_propagate(self._h, P, len(problems), E, len(ensembles),
                                              _ptr(stats_dev) if stats_dev is not None else None,
                                              _ptr(trace_dev) if trace_dev is not None else None,
                                              _stream(stream)))

    def match(self, problems, ensembles, maps_dev, dry_run=False, probe_dev=None, stream=None):
        P, E = self._arrays(problems, ensembles)
        self._check(lib().mcpr_reserve(self._h, P, len(problems), E, len(ensembles), RESERVE_MATCH))
        self._check(lib().mcpr_match(self._h, P, len(problems), E, len(ensembles), _ptr(maps_dev),
                                     1 if dry_run else 0,
                                     _ptr(probe_dev) if probe_dev is not None else None, _stream(stream)))


def fine_propagate_static(problems, ensembles, stats_dev=None, trace_dev=None, stream=None):
    """mcpr_fine_propagate_static: the fine propagator with its scratch in the
    library's static device array (no context, no allocation)."""
    L = lib()
    P = (ProblemC * len(problems))(*problems)
    E = (EnsembleC * len(ensembles))(*ensembles)
    st = L.mcpr_fine_propagate_static(P, len(problems), E, len(ensembles),
                                      _ptr(stats_dev) if stats_dev is not None else None,
                                      _ptr(trace_dev) if trace_dev is not None else None, _stream(stream))
    if st != 0:
        raise MCPRError(st, L.mcpr_last_error(None).decode())


def stream_probe(x, reps: int = 20, stream=None) -> float:
    """mcpr_stream_probe on a float32 device tensor (numel a multiple of
    4096): mean ms of one in-place streaming pass (8 bytes per float)."""
    L = lib()
    ms = ctypes.c_double()
    st = L.mcpr_stream_probe(_ptr(x), int(x.numel()), int(reps), _stream(stream), ctypes.byref(ms))
    if st != 0:
        raise MCPRError(st, L.mcpr_last_error(None).decode())
    return ms.value


def ensemble(x, instance=0, slice_index=0, problem=0, n=None) -> EnsembleC:
    e = EnsembleC()
    e.x = _ptr(x)
    e.n_particles = int(n if n is not None else x.numel())
    e.instance = int(instance)
    e.slice = int(slice_index)
    e.problem = int(problem)
    return e


def stats_buffer(n_ens: int, n_regions: int, device="cuda"):
    import torch
    return torch.empty(n_ens * (n_regions + 1) * STATS_DTYPE.itemsize, dtype=torch.uint8, device=device)


def stats_to_numpy(buf, n_ens: int, n_regions: int) -> np.ndarray:
    host = buf.cpu().numpy()[: n_ens * (n_regions + 1) * STATS_DTYPE.itemsize]
    return host.view(STATS_DTYPE).reshape(n_ens, n_regions + 1).copy()


def maps_to_device(maps: np.ndarray, device="cuda"):
    import torch
    arr = np.ascontiguousarray(maps, dtype=MAP_DTYPE)
    return torch.from_numpy(arr.view(np.uint8).copy()).to(device)


# ---------------------------------------------------------------------------
# convenience wrappers used by the tests and the benchmark
# ---------------------------------------------------------------------------
class Propagator:
    """Single-problem convenience layer over a Context."""

    def __init__(self, problem, ctx: Optional[Context] = None, coef=None):
        self.problem = problem
        self.pc = problem_c(problem, coef)
        self.ctx = ctx or Context(0)
        self.I = problem.n_regions

    def new_particles(self, P: int, device="cuda"):
        import torch
        return torch.empty(P, dtype=torch_dtype(self.problem.precision), device=device)

    def sample(self, x, instance=0):
        self.ctx.init_particles([self.pc], [ensemble(x, instance)])

    def moments(self, xs: List, instances=None) -> np.ndarray:
        inst = instances or [0] * len(xs)
        buf = stats_buffer(len(xs), self.I)
        self.ctx.moments([self.pc], [ensemble(x, i) for x, i in zip(xs, inst)], buf)
        return stats_to_numpy(buf, len(xs), self.I)

    def qoi(self, xs: List, kind: int = QOI_SIN_X2, instances=None) -> np.ndarray:
        import torch
        inst = instances or [0] * len(xs)
        out = torch.empty(len(xs), dtype=torch.float64, device=xs[0].device)
        self.ctx.qoi([self.pc], [ensemble(x, i) for x, i in zip(xs, inst)], kind, out)
        return out.cpu().numpy()

    def fine(self, xs: List, slices: Sequence[int], instances=None, trace=False):
        import torch
        inst = instances or [0] * len(xs)
        buf = stats_buffer(len(xs), self.I)
        tr = torch.empty(len(xs) * (self.problem.steps_per_slice + 1) * 2, dtype=torch.float64,
                         device="cuda") if trace else None
        self.ctx.fine_propagate([self.pc], [ensemble(x, i, n) for x, i, n in zip(xs, inst, slices)], buf, tr)
        st = stats_to_numpy(buf, len(xs), self.I)
        if trace:
            return st, tr.cpu().numpy().reshape(len(xs), self.problem.steps_per_slice + 1, 2)
        return st

    def match(self, xs: List, maps: np.ndarray, instances=None, dry_run=False):
        inst = instances or [0] * len(xs)
        dm = maps_to_device(maps)
        probe = stats_buffer(len(xs), self.I) if dry_run else None
        self.ctx.match([self.pc], [ensemble(x, i) for x, i in zip(xs, inst)], dm, dry_run, probe)
        if dry_run:
            return stats_to_numpy(probe, len(xs), self.I)
        return None


COEF_NAMES = ("a0", "a1", "a2", "a3", "am", "av", "b0", "b1", "bm", "bv")


def adjoint(ctx: Context, problem_struct: ProblemC, x0, dL_dmoments=None, instance=0, first_slice=0,
            stream=None):
    """Slice-end moments of the serial fine solution from x0 and, given
    dL/d(moments) [n, 2], the gradient dL/d(a0..bv) through mcpr_adjoint."""
    n = problem_struct.n_slices - first_slice
    mom = np.zeros((n, 2))
    e = ensemble(x0, instance, first_slice)
    P = (ProblemC * 1)(problem_struct)
    E = (EnsembleC * 1)(e)
    ctx._check(lib().mcpr_reserve(ctx.handle, P, 1, E, 1, RESERVE_ADJOINT))
    if dL_dmoments is None:
        ctx._check(lib().mcpr_adjoint(ctx.handle, P, E, None, mom.ctypes.data, None, _stream(stream)))
        return mom, None
    dl = np.ascontiguousarray(dL_dmoments, dtype=np.float64).reshape(n, 2)
    g = np.zeros(10)
    ctx._check(lib().mcpr_adjoint(ctx.handle, P, E, dl.ctypes.data, mom.ctypes.data, g.ctypes.data,
                                  _stream(stream)))
    return mom, g


def slice_moments_function():
    """torch.autograd.Function: coefficients (10, float64) -> slice-end
    (mean, variance) [N, 2] of the fine propagator; backward by the adjoint."""
    import torch

    class SliceMoments(torch.autograd.Function):
        @staticmethod
        def forward(fctx, coef, x0, problem, mctx, instance):
            pc = problem_c(problem, _coef_from(coef))
            mom, _ = adjoint(mctx, pc, x0, None, instance)
            fctx.save_for_backward(coef)
            fctx.x0, fctx.problem, fctx.mctx, fctx.instance = x0, problem, mctx, instance
            return torch.from_numpy(mom)

        @staticmethod
        def backward(fctx, grad_out):
            (coef,) = fctx.saved_tensors
            pc = problem_c(fctx.problem, _coef_from(coef))
            _, g = adjoint(fctx.mctx, pc, fctx.x0, grad_out.detach().cpu().numpy(), fctx.instance)
            return torch.from_numpy(g).to(coef.dtype), None, None, None, None

    return SliceMoments


def _coef_from(coef_tensor):
    from types import SimpleNamespace
    vals = [float(v) for v in coef_tensor.detach().cpu().tolist()]
    return SimpleNamespace(**dict(zip(COEF_NAMES, vals)))


class Parareal:
    """MC-moments Parareal over one or more instances (rings allocated here with torch)."""

    def __init__(self, problems: Sequence, P: Sequence[int], ctx: Optional[Context] = None,
                 coefs: Optional[Sequence] = None, instances: Optional[Sequence[int]] = None,
                 learning: bool = False, tol: float = 0.0, device="cuda"):
        import torch
        self.ctx = ctx or Context(0)
        self.problems = list(problems)
        n_inst = len(P)
        coefs = coefs or [None] * n_inst
        instances = instances if instances is not None else list(range(n_inst))
        pr0 = self.problems[0]
        self.N, self.I = pr0.n_slices, pr0.n_regions
        self.P = [int(p) for p in P]
        self.strides = [(p + 3) // 4 * 4 for p in self.P]
        dt = torch_dtype(pr0.precision)
        self.rings = [torch.empty((self.N + 1) * s, dtype=dt, device=device) for s in self.strides]
        self.pcs = [problem_c(self.problems[min(i, len(self.problems) - 1)], coefs[i]) for i in range(n_inst)]
        Pa = (ProblemC * n_inst)(*self.pcs)
        ins = (InstanceC * n_inst)()
        for i in range(n_inst):
            ins[i].problem = i
            ins[i].instance = int(instances[i])
            ins[i].n_particles = self.P[i]
            ins[i].slot_stride = self.strides[i]
            ins[i].ring = self.rings[i].data_ptr()
        h = ctypes.c_void_p()
        self.ctx._check(lib().mcpr_parareal_create(self.ctx.handle, Pa, n_inst, ins, n_inst,
                                                   1 if learning else 0, float(tol), ctypes.byref(h)))
        self._h = h
        self.n_inst = n_inst

    def close(self):
        if getattr(self, "_h", None):
            lib().mcpr_parareal_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, sample_u0=True, stream=None):
        self.ctx._check(lib().mcpr_parareal_init(self._h, 1 if sample_u0 else 0, _stream(stream)))

    def iterate(self, stream=None) -> np.ndarray:
        d = (ctypes.c_double * self.n_inst)()
        self.ctx._check(lib().mcpr_parareal_iterate(self._h, d, _stream(stream)))
        return np.array(d[:])

    @property
    def iteration(self) -> int:
        return int(lib().mcpr_parareal_iteration(self._h))

    def track_qoi(self, on: bool = True):
        """Record the QoI of each slice as it becomes exact (call before init)."""
        self.ctx._check(lib().mcpr_parareal_track_qoi(self._h, 1 if on else 0))

    def qoi(self, kind: int = QOI_SIN_X2, i: int = 0, stream=None) -> np.ndarray:
        """(1/P) sum Phi over u^k_n of instance i, n = 0..N."""
        out = np.zeros(self.N + 1)
        self.ctx._check(lib().mcpr_parareal_qoi(self._h, i, int(kind), out.ctypes.data, _stream(stream)))
        return out

    def set_fractions(self, fractions, i=0):
        """Given particle fractions [N+1, I] of every macro state of instance i
        (None: the method's own), from the next init or iterate on."""
        if fractions is None:
            self.ctx._check(lib().mcpr_parareal_set_fractions(self._h, i, None))
            return
        self._given = np.ascontiguousarray(fractions, dtype=np.float64).reshape(self.N + 1, self.I)
        self.ctx._check(lib().mcpr_parareal_set_fractions(self._h, i, self._given.ctypes.data))

    def macro(self, i=0):
        rho = np.zeros((self.N + 1, self.I, 3))
        glob = np.zeros((self.N + 1, 2))
        self.ctx._check(lib().mcpr_parareal_macro(self._h, i, rho.ctypes.data, glob.ctypes.data))
        return rho, glob

    def flags(self, i=0) -> np.ndarray:
        f = np.zeros((self.N, self.I), dtype=np.int32)
        self.ctx._check(lib().mcpr_parareal_flags(self._h, i, f.ctypes.data))
        return f

    def save(self) -> bytes:
        """The driver's host state (mcpr_parareal_save); the rings are the caller's."""
        n = ctypes.c_size_t()
        self.ctx._check(lib().mcpr_parareal_save(self._h, None, 0, ctypes.byref(n)))
        buf = (ctypes.c_char * n.value)()
        self.ctx._check(lib().mcpr_parareal_save(self._h, buf, n.value, ctypes.byref(n)))
        return bytes(buf)

    def restore(self, state: bytes):
        """mcpr_parareal_restore (copy the rings back first)."""
        buf = ctypes.create_string_buffer(state, len(state))
        self.ctx._check(lib().mcpr_parareal_restore(self._h, buf, len(state)))

    def slot(self, i: int, n: int):
        """Tensor view of u^k_n of instance i."""
        p = ctypes.c_void_p()
        self.ctx._check(lib().mcpr_parareal_slot(self._h, i, n, ctypes.byref(p)))
        esz = self.rings[i].element_size()
        off = (p.value - self.rings[i].data_ptr()) // esz
        return self.rings[i][off: off + self.P[i]]
