#!/usr/bin/env python3
"""Benchmark of the MC-moments Parareal hot path on one MI355X.

Default workload (the headline configuration, the largest that fits one
GPU): the bimodal Desai-Zwanzig ensemble dX = (X - X^3 - 0.5 (X - E[X])) dt
+ 0.5 dW, X0 ~ 0.5 N(-1, 0.1^2) + 0.5 N(1, 0.1^2), P = 1.6e7 particles per
slice, N = 256 slices propagated together (a 16.4 GB ring of fp32 states),
T = 10, dt = 5e-4 (79 steps per slice), two regions split at 0, the
particle-fraction learning model, tolerance 1e-4; fp32 particles with fp64
reductions and matching.

One step is one pass of the whole hot path over the workload's input: sample
p0, restriction, coarse sweep and lifting of all slices (iteration 0), then one
Parareal iteration: the fine propagator on every slice of every instance,
batched into each Euler-Maruyama launch, the slice-end restrictions, the
sequential coarse sweep with the iterator, and the matching.
value = particle-steps per second of the whole step.

Other workloads (--workload): dz_bimodal (P = 1e6, N = 50: a 204 MB ring that
fits the 256 MB Infinity Cache), ou_batched (64 independent OU instances, P
log-uniform in [1e4, 2e6], N = 32: 3.7 GB of state), ou_linear (P = 1e4,
N = 10, fp64: the latency-bound case), gbm (geometric Brownian motion with
interaction and multiplicative noise, P = 1e6, N = 10, fp32; the parareal
section adds the error of the QoI sin(X^2) of every slice against the serial
solution), burgers (the particle system of the viscous Burgers equation,
drift 1 - F_P(X) with the empirical CDF F_P, X(0) = 0, P = 1e6, N = 10, T = 1,
fp32: each Euler-Maruyama step ranks the ensemble; the roofline line then
covers the whole step sequence, sort included, against the same 8 B per
particle-step of state traffic), adjoint_ou / adjoint_dz (the gradient of the
slice-end moments' squared error through the fine propagator, P = 1e5, T = 2,
dt = 1e-3, N = 20, fp32 state: one step is one mcpr_adjoint call, i.e. the
forward solution with slice-start checkpoints, each slice recomputed, and the
backward sweep; value = forward particle-steps differentiated per second,
roofline = the backward step kernel, 20 B per particle-step: the state read,
the fp64 adjoint read and written).

The JSON line also carries:
  roofline      the Euler-Maruyama step kernel: algorithmic bytes per launch
                (8 B per particle-step in fp32, 16 B in fp64: one read and one
                write of the state) over its mean launch duration, measured
                with HIP events around each sweep's run of step launches inside
                the timed region, against 8 TB/s; bound "hbm" when the state
                ring exceeds the 256 MB Infinity Cache, else "mall"; traffic =
                HBM bytes per launch from rocprofv3 counters
                (profiles/traffic.json) while the kernel source is unchanged,
                else null;
  parareal      wall time of the serial fine solution against Parareal
                iterations on the same GPU; per iteration the largest error of
                the slice moments against the serial run, also in units of the
                Monte-Carlo standard error of each slice; the first iteration
                at equal accuracy (every slice within one standard error), the
                iteration reaching the tolerance, and the k = N run;
  precision     the fp32-state path against the fp64 oracle on one slice of
                the same law at P = 1e6 (default workload);
  fp64_per_slice  the plain fp64 per-slice GPU path (same kernels, fp64 state,
                one slice per call) on the same workload, and the speed-up of
                value over it (default workload);
  secondary     the 64-instance batch (3.7 GB, HBM-resident) measured the same
                way, and Parareal at equal accuracy on the latency-bound fp64
                case (default workload);
  cpu_baseline  the FP64 oracle on the host, one thread and all threads of the
                GPU's share of the host, on a bounded sample of the same
                workload (default workload).
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import math
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MALL_BYTES = 256 * 1024 * 1024  # MI355X Infinity Cache
DEFAULT_WORKLOAD = "dz_large"
# threads the host share of one GPU offers the CPU baseline (the boxes give a
# GPU's process 16 CPUs, whatever the machine's total)
CPU_SHARE = 16


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if any."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except Exception:
        return None
    ent = data.get(f"{kernel}@{workload}")
    if not ent:
        return None
    if ent.get("kernels_sha") != kernels_sha():
        return None  # the kernel changed since the counters were taken
    return ent.get("bytes_per_launch")


def kernels_sha() -> str:
    """Hash of the sources the Euler-Maruyama step kernels are built from
    (kernels, RNG, shared types)."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "rng.hpp", "common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2310_11365_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def host_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def make_workload(name: str, particles: int = 0):
    """(workload, per-instance particle counts, coefficient overrides, description).
    particles > 0 replaces the particle count of a one-instance workload."""
    from paper_2310_11365_amd import workloads as W
    if particles > 0:
        if name == "ou_batched":
            raise SystemExit("--particles applies to one-instance workloads")
        wl, _, coefs, desc = make_workload(name)
        wl = dataclasses.replace(wl, P=particles)
        return wl, [particles], coefs, desc + f"; particle count replaced: P={particles}"
    if name == "dz_bimodal":
        wl = W.dz_bimodal()
        return wl, [wl.P], None, ("dz_bimodal: Desai-Zwanzig dX=(X-X^3-0.5(X-E[X]))dt+0.5dW, "
                                  "X0~0.5N(-1,0.1^2)+0.5N(1,0.1^2), P=1e6, N=50, T=5, two regions split at 0")
    if name == "ou_batched":
        wl = W.ou_batched()
        return wl, [i["P"] for i in wl.instances], [i["coef"] for i in wl.instances], \
            ("ou_batched: 64 independent instances of dX=(-theta X+0.5E[X])dt+sigma dW, X0~N(1,0.2^2), "
             "theta~U[0.1,1], sigma~U[0.2,0.8], P log-uniform in [1e4,2e6], N=32")
    if name == "dz_large":
        wl = W.dz_large()
        return wl, [wl.P], None, ("dz_large: Desai-Zwanzig dX=(X-X^3-0.5(X-E[X]))dt+0.5dW, "
                                  "X0~0.5N(-1,0.1^2)+0.5N(1,0.1^2), two regions split at 0, P=1.6e7, N=256, "
                                  "T=10, dt=5e-4 (79 steps per slice), fraction-model learning, tol 1e-4")
    if name == "gbm":
        wl = W.gbm(P=1_000_000, precision=W.FP32)
        return wl, [wl.P], None, ("gbm: dX=(-X/2+0.8E[X]+1/3)dt+(s X+s E[X]+1/6)dW, s=sqrt(1/8), X0~N(1,1/4), "
                                  "P=1e6, T=1, N=10, QoI sin(X^2)")
    if name == "burgers":
        wl = W.burgers(P=1_000_000, precision=W.FP32)
        return wl, [wl.P], None, ("burgers: dX=(1-F_P(X))dt+dW, F_P the empirical CDF with H(0)=1/2, X0=0, "
                                  "P=1e6, T=1, N=10; the ensemble ranked every step")
    if name == "ou_linear":
        wl = W.ou_linear()
        return wl, [wl.P], None, ("ou_linear: dX=(-X+0.5E[X])dt+0.3dW, X0~N(1,0.2^2), P=1e4, N=10, "
                                  "RK4 coarse h=0.05, fp64")
    raise SystemExit(f"unknown workload {name}")


# ---------------------------------------------------------------------------
# CPU baseline: the oracle as it stands, on a bounded sample of the workload
# ---------------------------------------------------------------------------
def oracle_worker(workload: str, slice_index: int, steps: int):
    """Child process: the oracle's fine propagator (fp64, one thread) for
    `steps` Euler-Maruyama steps of one slice at the workload's full particle
    count; prints {"ps", "seconds"} as JSON.  Imports no GPU code."""
    from oracle import oracle as O
    from paper_2310_11365_amd import workloads as W
    wl, sizes, _, _ = make_workload(workload)
    pr = dataclasses.replace(wl.problem, precision=W.FP64, steps_per_slice=steps)
    x = O.sample_p0(pr, sizes[0])
    t0 = time.perf_counter()
    O.fine(pr, x, slice_index)
    dt = time.perf_counter() - t0
    print(json.dumps({"ps": sizes[0] * steps, "seconds": dt}), flush=True)


def cpu_baseline(workload: str, steps: int):
    """One oracle process, then one per thread of the host share, each
    running `steps` steps of its own slice at full size; particle-steps/s of
    each run (all processes together for the second)."""
    from oracle import oracle as O
    if not os.path.exists(O.LIB):
        O.build(force=False)

    def run(nproc):
        procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker",
                                   "--workload", workload, "--worker-slice", str(i), "--worker-steps", str(steps)],
                                  stdout=subprocess.PIPE, text=True, cwd=ROOT) for i in range(nproc)]
        t0 = time.perf_counter()
        res = []
        for p in procs:
            out, _ = p.communicate(timeout=600)
            if p.returncode != 0:
                raise RuntimeError("oracle worker failed")
            res.append(json.loads(out.strip().splitlines()[-1]))
        wall = time.perf_counter() - t0
        return res, wall

    one, _ = run(1)
    nthr = max(1, min(CPU_SHARE, host_threads()))
    many, _ = run(nthr)
    v1 = one[0]["ps"] / one[0]["seconds"]
    # all processes run at once: aggregate rate = total work / longest run
    vn = sum(r["ps"] for r in many) / max(r["seconds"] for r in many)
    P = one[0]["ps"] // steps
    return {"value": vn, "unit": "particle-steps/s", "cores": nthr, "kind": "oracle",
            "sample": f"{steps} Euler-Maruyama steps of one slice at the workload's full size (P={P}) in fp64, "
                      f"one oracle process per thread, {nthr} at once, each on its own slice "
                      f"({sum(r['ps'] for r in many):.3g} particle-steps, longest {max(r['seconds'] for r in many):.1f} s)",
            "single_thread": {"value": v1, "cores": 1, "seconds": one[0]["seconds"]},
            "host": {"cpu_model": cpu_model(), "nproc": os.cpu_count(), "threads_available": host_threads()}}


# ---------------------------------------------------------------------------
# GPU measurements
# ---------------------------------------------------------------------------
def throughput(name: str, steps: int, warmup: int, variant: int, particles: int = 0):
    """Whole hot-path steps (init + one iteration) of a workload: wall clock
    over the timed steps, and the step kernel's mean launch time by HIP
    events inside the timed region.  A context of its own, so that its
    autotuner holds the one launch shape of these steps."""
    import torch

    from paper_2310_11365_amd import mcpr
    from paper_2310_11365_amd import workloads as W
    wl, sizes, coefs, desc = make_workload(name, particles)
    pr = wl.problem
    N, m = pr.n_slices, pr.steps_per_slice
    ps_per_step = N * m * sum(sizes)
    esize = 8 if pr.precision == W.FP64 else 4
    tname = "double" if pr.precision == W.FP64 else "float"
    ctx = mcpr.Context(0)
    ctx.set_tuning(variant)
    para = mcpr.Parareal([pr], sizes, ctx, coefs=coefs, learning=wl.learning, tol=wl.tol)

    def step():
        para.init()
        para.iterate()

    print(f"# workload {wl.name}: {len(sizes)} instance(s), {sum(sizes)} particles per slice in total, "
          f"N={N} m={m}; warmup {warmup}", flush=True)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step()
        print(f"# {wl.name} step {i + 1}/{steps} done", flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    em_ms, em_launches, em_ps = ctx.profile_read(reset=True)
    ctx.profile(False)
    tv = ctx.tuned_variants()
    resident = ctx.resident_sweeps() > 0
    para.close()
    del para
    ctx.close()

    value = ps_per_step * steps / elapsed
    avg_launch_s = em_ms / 1e3 / max(em_launches, 1)
    bytes_per_launch = 2.0 * esize * (em_ps / max(em_launches, 1))  # one read and one write of the state
    achieved = bytes_per_launch / avg_launch_s / 1e9
    all_coefs = coefs if coefs else [pr.coef]
    deg = 1 if all(c.a2 == 0.0 and c.a3 == 0.0 for c in all_coefs) else 3
    v = variant if variant >= 0 else (tv[0] if len(tv) == 1 else -1)
    kernel = f"k_em_step<{tname}, {deg}, {'true' if v & 1 else 'false'}, {'true' if v & 2 else 'false'}>"
    if resident:
        kernel = (f"resident sweep: k_sweep_normals<{tname}> (every step's normals) + "
                  f"k_em_sweep_resident<{tname}, {deg}> (one block per ensemble through all the steps)")
        v = -1
    if pr.coef.acdf != 0.0:
        kernel = (f"empirical-CDF step sequence (library radix sort on a sweep's first steps, then buckets: "
                  f"k_combine, k_em_step_sorted<{tname}, {deg}, false>, k_cdf_bscan, k_cdf_bsort<{tname}>)")
    state_bytes = (N + 1) * sum((P + 3) // 4 * 4 for P in sizes) * esize
    roofline = {"bound": "hbm" if state_bytes > MALL_BYTES else "mall", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": load_traffic(kernel, wl.name), "kernel": kernel,
                "avg_launch_us": round(avg_launch_s * 1e6, 2), "launches": em_launches,
                "particle_steps_per_launch": em_ps / max(em_launches, 1), "bytes_per_launch": bytes_per_launch,
                "step_variant": v}
    if state_bytes <= MALL_BYTES:
        roofline["note"] = (f"the {state_bytes / 1e6:.0f} MB ring fits the 256 MB Infinity Cache, so the step "
                            f"streams from it rather than from HBM; the fraction is still taken against 8 TB/s")
    res = {"value": value, "ms_per_step": elapsed / steps * 1e3, "steps": steps, "warmup": warmup,
           "dtype": "f64" if pr.precision == W.FP64 else "f32 state / f64 reductions and matching",
           "config": {"workload": desc, "instances": len(sizes), "particles_per_slice": sum(sizes),
                      "slices": N, "steps_per_slice": m, "dt": pr.dt, "state_bytes": state_bytes,
                      "particle_steps_per_step": ps_per_step,
                      "step": "iteration 0 (sample, restrict, coarse, lift) + one Parareal iteration over "
                              "all slices"},
           "roofline": roofline}
    return res


def parareal_section(ctx, name: str, max_s: float, max_iters: int = 0):
    """Serial fine solution vs Parareal iterations on the same GPU, errors
    in units of each slice's Monte-Carlo standard error."""
    import numpy as np
    import torch

    from paper_2310_11365_amd import mcpr
    wl, sizes, coefs, _ = make_workload(name)
    pr = wl.problem
    N, I = pr.n_slices, pr.n_regions
    n_inst = len(sizes)
    pcs = [mcpr.problem_c(pr, coefs[i] if coefs else None) for i in range(n_inst)]
    xs = [torch.empty(P, dtype=mcpr.torch_dtype(pr.precision), device="cuda") for P in sizes]
    ens = lambda n: [mcpr.ensemble(x, i, n, i) for i, x in enumerate(xs)]  # noqa: E731
    qoi_kind = mcpr.QOI_SIN_X2 if wl.name == "gbm" else None
    qbuf = torch.empty(n_inst, dtype=torch.float64, device="cuda")
    buf = mcpr.stats_buffer(n_inst, I)

    def serial(measure):
        """The serial run (timed unless measure: then the fourth central
        moment of each slice is taken along, for the standard error of V)."""
        ser, ser_q, mu4 = [], [], []
        ctx.init_particles(pcs, ens(0))
        for n in range(N + 1):
            if n > 0:
                ctx.fine_propagate(pcs, ens(n - 1), buf)
            else:
                ctx.moments(pcs, ens(0), buf)
            ser.append(mcpr.stats_to_numpy(buf, n_inst, I))
            if qoi_kind is not None and not measure:
                ctx.qoi(pcs, ens(n), qoi_kind, qbuf)
                ser_q.append(qbuf.cpu().numpy().copy())
            if measure:
                row = []
                for x in xs:
                    d = x.double()
                    d -= d.mean()
                    row.append(float((d * d * d * d).mean()))
                mu4.append(row)
        return ser, ser_q, mu4

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ser, ser_q, _ = serial(False)
    torch.cuda.synchronize()
    t_serial = time.perf_counter() - t0
    _, _, mu4 = serial(True)
    del xs
    sm = np.array([[r[i][-1]["mean"] for r in ser] for i in range(n_inst)])  # [inst, N+1]
    sv = np.array([[r[i][-1]["var"] for r in ser] for i in range(n_inst)])
    m4 = np.array(mu4).T
    P = np.array(sizes, dtype=np.float64)[:, None]
    se_m = np.sqrt(sv / P)
    se_v = np.sqrt(np.maximum(m4 - sv * sv, 0.0) / P)

    # tol 0: the driver keeps iterating past the tolerance (the iterates do
    # not depend on it), so one run gives the iteration at the tolerance and
    # the run to k = N
    para = mcpr.Parareal([pr], sizes, ctx, coefs=coefs, learning=wl.learning, tol=0.0)
    if qoi_kind is not None:
        para.track_qoi(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    para.init()
    kmax = max_iters if max_iters > 0 else N
    rec = {"k": [], "wall_s": [], "delta": [], "E_mean": [], "E_var": [], "E_mean_over_se": [], "E_var_over_se": []}
    if qoi_kind is not None:
        rec["E_qoi"] = []
    k_tol = k_eq = None
    capped = False
    for k in range(kmax):
        delta = para.iterate()
        wall = time.perf_counter() - t0
        em = ev = rm = rv = 0.0
        for i in range(n_inst):
            _, glob = para.macro(i)
            dm, dv = np.abs(glob[:, 0] - sm[i]), np.abs(glob[:, 1] - sv[i])
            em, ev = max(em, float(dm.max())), max(ev, float(dv.max()))
            rm = max(rm, float(np.max(dm[1:] / se_m[i, 1:])))
            rv = max(rv, float(np.max(dv[1:] / np.maximum(se_v[i, 1:], 1e-300))))
        for key, val in (("k", k + 1), ("wall_s", round(wall, 4)), ("delta", float(np.max(delta))),
                         ("E_mean", em), ("E_var", ev), ("E_mean_over_se", round(rm, 4)),
                         ("E_var_over_se", round(rv, 4))):
            rec[key].append(val)
        if qoi_kind is not None:
            sq = np.array(ser_q)
            rec["E_qoi"].append(max(float(np.max(np.abs(para.qoi(qoi_kind, i) - sq[:, i]))) for i in range(n_inst)))
        if k_eq is None and rm <= 1.0 and rv <= 1.0:
            k_eq = k + 1
        if (k + 1) % 16 == 0 or k < 4 or k_eq == k + 1:
            print(f"# {wl.name} parareal k={k + 1} delta={np.max(delta):.3e} E_mean={em:.3e} ({rm:.2f} se) "
                  f"E_var={ev:.3e} ({rv:.2f} se) {wall:.2f} s", flush=True)
        if wl.tol > 0 and k_tol is None and np.max(delta) <= wl.tol:
            k_tol = k + 1
        if para.iteration >= N:
            break
        if wall > max_s:
            capped = True
            print(f"# {wl.name} parareal: time cap of {max_s} s reached at k={k + 1}", flush=True)
            break
    para.close()

    def at(k):
        return None if k is None else {"k": k, "wall_s": rec["wall_s"][k - 1],
                                       "speedup_vs_serial": round(t_serial / rec["wall_s"][k - 1], 4)}
    out = {"serial_s": round(t_serial, 4), "tol": wl.tol, "iterations": rec,
           "mc_standard_error": {"mean_max": float(se_m[:, 1:].max()), "var_max": float(se_v[:, 1:].max()),
                                 "definition": "se(M_n) = sqrt(V_n / P), se(V_n) = sqrt((mu4_n - V_n^2) / P) of the "
                                               "serial run's slice n"},
           "equal_accuracy": at(k_eq), "at_tol": at(k_tol),
           "at_k_equal_N": at(rec["k"][-1]) if rec["k"] and rec["k"][-1] >= N else None,
           "time_capped": capped,
           "note": "E_mean, E_var: largest error of the global slice moments against the serial fine solution "
                   "with the same random numbers; equal_accuracy: the first iteration at which every slice is "
                   "within one Monte-Carlo standard error of it. On one GPU an iteration's sweep over the "
                   "remaining slices moves as many bytes as the serial solve when the state streams from HBM, so "
                   "Parareal gains only at latency-bound sizes; across GPUs the sweep shards by slices."}
    if wl.tol > 0:
        out["tol_vs_se"] = (f"tol {wl.tol:g} against se(M) up to {se_m[:, 1:].max():.2e}: "
                            + ("below" if wl.tol < se_m[:, 1:].max() else "above") + " the standard error")
    return out


def precision_section(ctx, P: int = 1_000_000):
    """fp32 state (fp64 reductions) against the fp64 oracle: one slice of the
    default workload's law at P particles."""
    import torch

    from oracle import oracle as O
    from paper_2310_11365_amd import mcpr
    from paper_2310_11365_amd import workloads as W
    wl, _, _, _ = make_workload(DEFAULT_WORKLOAD)
    pr = wl.problem
    pr64 = dataclasses.replace(pr, precision=W.FP64)
    prop = mcpr.Propagator(pr, ctx)
    x = prop.new_particles(P)
    prop.sample(x)
    g = prop.fine([x], [0])[0]
    del x
    torch.cuda.synchronize()
    o = O.restrict(pr64, O.fine(pr64, O.sample_p0(pr64, P), 0)[0])
    wm = wv = 0.0
    for i in range(len(o)):
        sc = abs(o[i]["mean"]) + math.sqrt(o[i]["var"])
        wm = max(wm, abs(g[i]["mean"] - o[i]["mean"]) / sc)
        wv = max(wv, abs(g[i]["var"] - o[i]["var"]) / o[i]["var"])
    return {"sample": f"slice 0 ({pr.steps_per_slice} steps) of the default workload's law at P={P}",
            "mean_err_over_abs_m_plus_sd": wm, "var_rel_err": wv,
            "tested_bound": {"mean": 2e-5, "var": 2e-4},
            "mc_standard_error_of_mean_at_full_size": math.sqrt(float(o[-1]["var"]) / wl.P),
            "reductions": "every sum over particles is fp64 from the particle up (d = x - shift formed in fp64); "
                          "the step kernel's sums of a 1.6e7-particle fp32 state agree with long-double moments "
                          "of the same values to 1e-13 (GPU test)"}


def fp64_per_slice(ctx, name: str, n_slices: int):
    """The plain fp64 per-slice GPU path: fp64 state, one slice per call,
    slices in sequence (no batching across slices)."""
    import torch

    from paper_2310_11365_amd import mcpr
    from paper_2310_11365_amd import workloads as W
    wl, sizes, _, _ = make_workload(name)
    pr64 = dataclasses.replace(wl.problem, precision=W.FP64)
    pc64 = mcpr.problem_c(pr64)
    x64 = torch.empty(sizes[0], dtype=torch.float64, device="cuda")
    ctx.init_particles([pc64], [mcpr.ensemble(x64, 0)])
    buf = mcpr.stats_buffer(1, pr64.n_regions)
    ctx.fine_propagate([pc64], [mcpr.ensemble(x64, 0, 0)], buf)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(1, n_slices + 1):
        ctx.fine_propagate([pc64], [mcpr.ensemble(x64, 0, n)], buf)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    del x64
    return n_slices * pr64.steps_per_slice * sizes[0] / t64


def bench_adjoint(args):
    import numpy as np
    import torch

    from paper_2310_11365_amd import mcpr
    from paper_2310_11365_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    kind = args.workload.split("_", 1)[1]
    wl = W.adjoint_case(kind, precision=W.FP32)
    pr, P = wl.problem, wl.P
    N, m = pr.n_slices, pr.steps_per_slice
    ctx = mcpr.Context(0)
    ctx.set_tuning(args.variant)
    prop = mcpr.Propagator(pr, ctx)
    x = prop.new_particles(P)
    prop.sample(x)
    pc = mcpr.problem_c(pr)
    # targets: the slice-end moments at every coefficient scaled by 1.1, same noise
    coef_t = W.Coef(*[1.1 * c for c in pr.coef.as_list()])
    tgt, _ = mcpr.adjoint(ctx, mcpr.problem_c(pr, coef_t), x)
    mom, _ = mcpr.adjoint(ctx, pc, x)
    dl = 2.0 * (mom - tgt)
    J = float(np.sum((mom - tgt) ** 2))

    print(f"# workload {wl.name}: P={P} N={N} m={m}; warmup {args.warmup}", flush=True)
    for _ in range(args.warmup):
        mcpr.adjoint(ctx, pc, x, dl)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read_adjoint(reset=True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, g = mcpr.adjoint(ctx, pc, x, dl)
        print(f"# step {i + 1}/{args.steps} done", flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    adj_ms, adj_steps, adj_ps = ctx.profile_read_adjoint(reset=True)
    ctx.profile(False)

    ps_per_step = N * m * P
    avg_s = adj_ms / 1e3 / max(adj_steps, 1)
    bytes_per_launch = 20.0 * adj_ps / max(adj_steps, 1)
    achieved = bytes_per_launch / avg_s / 1e9
    nsc = -(-((P + 3) // 4) // (256 * (1 if P < 65536 else 4)))
    kernel = f"k_adj_step<float, {'true' if nsc > 256 else 'false'}>"
    out = {"metric": "fine-propagator particle-steps/sec", "value": ps_per_step * args.steps / elapsed,
           "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32 state / f64 adjoint and reductions", "data": "synthetic",
           "config": {"workload": f"{wl.name}: gradient of sum_n (m_n - M_n)^2 + (v_n - V_n)^2 with respect to "
                                  f"the ten drift and diffusion coefficients, targets at 1.1x the coefficients",
                      "instances": 1, "particles_per_slice": P, "slices": N, "steps_per_slice": m, "dt": pr.dt,
                      "particle_steps_per_step": ps_per_step,
                      "step": "one adjoint call: forward with slice checkpoints, per-slice recomputation, "
                              "backward sweep", "J": J, "grad_norm": float(np.linalg.norm(g))},
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": kernel,
                        "avg_launch_us": round(avg_s * 1e6, 2), "bytes_per_launch": bytes_per_launch,
                        "note": "1e5 particles: launch-latency bound, far from the HBM roof"}}
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD,
                    choices=["dz_large", "dz_bimodal", "ou_batched", "ou_linear", "gbm", "burgers", "adjoint_ou",
                             "adjoint_dz"])
    ap.add_argument("--particles", type=int, default=0,
                    help="replace the particle count of a one-instance workload (e.g. to move its ring across "
                         "the Infinity Cache size)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parareal", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="default workload: skip the batched-OU line, the fp64 Parareal case, the precision "
                         "check and the fp64 per-slice path")
    ap.add_argument("--parareal-iters", type=int, default=0,
                    help="Parareal iterations of the parareal section (0: up to N, the tolerance or the time cap)")
    ap.add_argument("--parareal-max-s", type=float, default=90.0,
                    help="stop the Parareal measurement after this many seconds")
    ap.add_argument("--cpu-steps", type=int, default=8,
                    help="Euler-Maruyama steps per oracle process in the CPU baseline")
    ap.add_argument("--variant", type=int, default=-1, choices=list(range(-1, 4)),
                    help="step-kernel launch variant: -1 autotune (default), 0..3 force (bit 0 non-temporal, "
                         "bit 1 separate mean-field combine)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MiB",
                    help="first run one plain device-to-device copy of this many MiB (a known-size "
                         "reference for the HBM byte counters of a profiler run)")
    ap.add_argument("--oracle-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--worker-slice", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--worker-steps", type=int, default=16, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_worker:
        return oracle_worker(args.workload, args.worker_slice, args.worker_steps)
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (the fine sweep would shard by slice "
              "ranges across GPUs; that exchange is not implemented); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.workload.startswith("adjoint_"):
        return bench_adjoint(args)

    default = args.workload == DEFAULT_WORKLOAD and args.particles == 0
    cpu = None
    if default and not args.no_cpu_baseline:
        # first, before this process touches the GPU: the oracle runs in child processes
        cpu = cpu_baseline(args.workload, args.cpu_steps)
        print(f"# cpu baseline: {cpu['value']:.3e} particle-steps/s on {cpu['cores']} threads, "
              f"{cpu['single_thread']['value']:.3e} on one", flush=True)

    import torch

    from paper_2310_11365_amd import mcpr

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.copy_probe > 0:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy probe: {n * 4} bytes read, {n * 4} bytes written", flush=True)
        del src, dst

    main_res = throughput(args.workload, args.steps, args.warmup, args.variant, args.particles)
    if main_res["roofline"]["bound"] == "hbm":
        # what the memory system sustains for the step kernel's access pattern
        # over as many bytes as the ring (in-place read and write, no arithmetic)
        n = main_res["config"]["state_bytes"] // 4 // 4096 * 4096
        probe = torch.ones(n, dtype=torch.float32, device="cuda")
        ms = mcpr.stream_probe(probe, 20)
        del probe
        ceil = 8.0 * n / (ms / 1e3) / 1e9
        main_res["roofline"]["stream_ceiling"] = {
            "achieved": round(ceil, 1), "unit": "GB/s", "frac_of_peak": round(ceil / HBM_PEAK_GBS, 4),
            "kernel_frac_of_ceiling": round(main_res["roofline"]["achieved"] / ceil, 4),
            "what": f"mcpr_stream_probe: in-place read and write of {8 * n / 1e9:.3g} GB with the step kernel's "
                    f"block shape and non-temporal access, no arithmetic (mean of 20 passes)"}
        print(f"# stream ceiling {ceil:.1f} GB/s", flush=True)
    out = {"metric": "fine-propagator particle-steps/sec", "value": main_res["value"], "unit": "particle-steps/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_res["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": main_res["dtype"],
           "data": "synthetic", "config": main_res["config"], "roofline": main_res["roofline"]}

    ctx = mcpr.Context(0)
    if not args.no_parareal and args.particles == 0:
        out["parareal"] = parareal_section(ctx, args.workload, args.parareal_max_s, args.parareal_iters)

    if default and not args.no_secondary:
        prec = precision_section(ctx)
        out["precision"] = prec
        print(f"# precision: fp32 vs fp64 oracle mean {prec['mean_err_over_abs_m_plus_sd']:.2e}, "
              f"var {prec['var_rel_err']:.2e}", flush=True)
        v64 = fp64_per_slice(ctx, args.workload, 8)
        out["fp64_per_slice"] = {
            "value": v64, "unit": "particle-steps/s", "speedup_of_value": out["value"] / v64,
            "sample": "slices 1..8 of the same workload in fp64, one slice per call",
            "equal_accuracy": (f"the fp32-state error against the fp64 oracle (precision section: "
                               f"{prec['mean_err_over_abs_m_plus_sd']:.1e} on the mean) against the Monte-Carlo "
                               f"standard error of the mean at full size "
                               f"({prec['mc_standard_error_of_mean_at_full_size']:.1e})")}
        print(f"# fp64 per-slice path {v64:.3e} particle-steps/s", flush=True)
        sec = throughput("ou_batched", 5, 1, -1)
        out["secondary"] = {
            "ou_batched": {"value": sec["value"], "unit": "particle-steps/s", "ms_per_step": sec["ms_per_step"],
                           "steps": 5, "warmup": 1, "config": sec["config"], "roofline": sec["roofline"]},
            "ou_linear_parareal": parareal_section(ctx, "ou_linear", 30.0)}
        print(f"# secondary ou_batched {sec['value']:.3e} particle-steps/s, frac {sec['roofline']['frac']}",
              flush=True)
    ctx.close()
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
