#!/usr/bin/env python3
"""Benchmark of the MC-moments Parareal hot path on one MI355X.

Workload: the bimodal Desai-Zwanzig ensemble (P = 1e6 particles per slice,
N = 50 slices, T = 5, dt = 1e-3, two regions split at 0, fp32 particles with
fp64 reductions and matching).  One step is one pass of the whole hot path
over that input: sample p0, restriction, coarse sweep and lifting of all 50
slices (iteration 0), then one Parareal iteration: the fine propagator on all
50 slices batched into each Euler-Maruyama launch (5e9 particle-steps),
slice-end restrictions, the sequential coarse sweep with the iterator, and
the matching.  value = particle-steps per second of the whole step.

The JSON line also carries:
  roofline      the Euler-Maruyama step kernel: algorithmic bytes per launch
                (8 B per particle-step: one fp32 read and one fp32 write) over
                its average launch duration, measured with HIP events around
                every step launch of the timed region, against 8 TB/s;
  cpu_baseline  the FP64 oracle on this host (one thread) on a bounded sample
                of the same workload;
  parareal      wall-time of the serial fine solution vs Parareal iterations
                on the same GPU, with the error of each iterate against the
                serial solution.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def load_traffic(kernel: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if any."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except Exception:
        return None
    ent = data.get(kernel)
    if not ent:
        return None
    lib = os.path.join(ROOT, "paper_2310_11365_amd", "csrc", "kernels.hip")
    import hashlib
    h = hashlib.sha256(open(lib, "rb").read()).hexdigest()[:16]
    if ent.get("kernels_sha") != h:
        return None  # the kernel changed since the counters were taken
    return ent.get("bytes_per_launch")


def cpu_baseline(seconds_target: float = 15.0):
    """The oracle as it stands (one thread) on whole slices of the workload at
    P = 1e6 in fp64, slice after slice until about seconds_target."""
    from oracle import oracle as O
    from paper_2310_11365_amd import workloads as W
    if not os.path.exists(O.LIB):
        O.build(force=False)
    wl = W.dz_bimodal(precision=W.FP64)
    pr, P = wl.problem, wl.P
    x = O.sample_p0(pr, P)
    t0 = time.perf_counter()
    slices = 0
    while slices < pr.n_slices:
        x, _ = O.fine(pr, x, slices)
        slices += 1
        if time.perf_counter() - t0 >= seconds_target:
            break
    dt = time.perf_counter() - t0
    ps = P * pr.steps_per_slice * slices
    return {"value": ps / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"bimodal workload at fp64, P={P}, serial fine solution of slices 0..{slices - 1} "
                      f"({ps:.3g} particle-steps), single thread, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parareal", action="store_true")
    ap.add_argument("--parareal-iters", type=int, default=4)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MiB",
                    help="first run one plain device-to-device copy of this many MiB (a known-size "
                         "reference for the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (slice sharding across GPUs is "
              "described in DESIGN.md but not implemented); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2310_11365_amd import mcpr
    from paper_2310_11365_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = W.dz_bimodal()
    pr = wl.problem
    N, m, P = pr.n_slices, pr.steps_per_slice, wl.P
    ps_per_step = N * m * P

    if args.copy_probe > 0:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy probe: {n * 4} bytes read, {n * 4} bytes written", flush=True)
        del src, dst

    ctx = mcpr.Context(0)
    para = mcpr.Parareal([pr], [P], ctx)

    def step():
        para.init()
        para.iterate()

    print(f"# workload {wl.name}: P={P} N={N} m={m} fp32/fp64-reduce; warmup {args.warmup}", flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        print(f"# step {i + 1}/{args.steps} done", flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    em_ms, em_launches, em_ps = ctx.profile_read(reset=True)
    ctx.profile(False)

    value = ps_per_step * args.steps / elapsed
    avg_launch_s = em_ms / 1e3 / max(em_launches, 1)
    bytes_per_launch = 8.0 * (em_ps / max(em_launches, 1))  # fp32 read + write per particle-step
    achieved = bytes_per_launch / avg_launch_s / 1e9
    traffic = load_traffic("k_em_step<float>")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_em_step<float>", "avg_launch_us": round(avg_launch_s * 1e6, 2),
                "bytes_per_launch": bytes_per_launch}

    out = {"metric": "fine-propagator particle-steps/sec", "value": value, "unit": "particle-steps/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32 state / f64 reductions", "data": "synthetic",
           "config": {"workload": "dz_bimodal: Desai-Zwanzig dX=(X-X^3-0.5(X-E[X]))dt+0.5dW, "
                                  "X0~0.5N(-1,0.1^2)+0.5N(1,0.1^2), two regions split at 0",
                      "particles": P, "slices": N, "steps_per_slice": m, "T": 5.0, "dt": pr.dt,
                      "particle_steps_per_step": ps_per_step,
                      "step": "iteration 0 (sample, restrict, coarse, lift) + one Parareal iteration "
                              "over all slices"},
           "roofline": roofline}

    if not args.no_parareal:
        # serial fine solution vs Parareal iterations, same GPU, same kernels
        prop = mcpr.Propagator(pr, ctx)
        x = prop.new_particles(P)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prop.sample(x)
        ser = [prop.moments([x])[0]]
        for n in range(N):
            ser.append(prop.fine([x], [n])[0])
        torch.cuda.synchronize()
        t_serial = time.perf_counter() - t0
        sm = np.array([r[-1]["mean"] for r in ser])
        sv = np.array([r[-1]["var"] for r in ser])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        para.init()
        it = []
        for k in range(args.parareal_iters):
            para.iterate()
            _, glob = para.macro(0)
            it.append({"k": k + 1, "wall_s": round(time.perf_counter() - t0, 4),
                       "E_mean": float(np.max(np.abs(glob[:, 0] - sm))),
                       "E_var": float(np.max(np.abs(glob[:, 1] - sv)))})
        se_mean = math.sqrt(float(np.max(sv)) / P)
        out["parareal"] = {"serial_s": round(t_serial, 4), "iterations": it,
                           "mc_standard_error_mean": se_mean,
                           "note": "one GPU: the fine sweep of an iteration moves as many bytes as the "
                                   "serial run, so iterations cost about as much as the serial solve"}

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()

    para.close()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
