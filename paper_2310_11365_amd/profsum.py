"""Summaries of rocprofv3 output databases (kernel traces and byte counters).

Reads the SQLite databases rocprofv3 writes (-d DIR -o run) and prints the
per-kernel statistics and the HBM byte counts per dispatch, scaled by the
reading of a plain device copy of known size (bench.py --copy-probe).  Used to
write the summaries kept under profiles/.

    python -m paper_2310_11365_amd.profsum trace DB [--bench-log LOG]
    python -m paper_2310_11365_amd.profsum traffic FETCH_DB WRITE_DB --kernel NAME --copy-mib 1024
    python -m paper_2310_11365_amd.profsum valu DB --kernel NAME --trace-us MEAN_US
"""
from __future__ import annotations

import argparse
import json
import sqlite3
import statistics


def short_name(name: str) -> str:
    """Kernel name without its argument list, 'void ' and anonymous namespaces."""
    name = name.replace("(anonymous namespace)::", "").replace("ROCPRIM_400200_NS::detail::", "")
    return name.split("(")[0].replace("void ", "")


def kernel_table(db_path: str, limit: int = 12):
    cur = sqlite3.connect(db_path).cursor()
    rows = list(cur.execute("select name, total_calls, total_duration, average, percentage from top_kernels "
                            "order by total_duration desc limit ?", (limit,)))
    return [(short_name(r[0]), int(r[1]), float(r[2]), float(r[3]), float(r[4])) for r in rows]


def grid_column(cur):
    """Name of the kernels view's column holding the grid's x extent (in work items)."""
    cols = [r[1] for r in cur.execute("pragma table_info(kernels)")]
    for c in cols:
        lc = c.lower()
        if "grid" in lc and lc.endswith("x"):
            return c
    return None


def durations(db_path: str, kernel: str, grid=None):
    """Durations (us) of every dispatch of kernel; grid: only dispatches with
    that x extent of the grid (work items)."""
    cur = sqlite3.connect(db_path).cursor()
    gc = grid_column(cur)
    out = []
    q = f"select name, duration, {gc} from kernels" if gc else "select name, duration, 0 from kernels"
    for name, d, g in cur.execute(q):
        if short_name(name).replace("mcpr::", "") == kernel and (grid is None or int(g) == grid):
            out.append(d / 1e3)
    return out


def grid_groups(db_path: str, kernel: str):
    """{grid x extent: dispatch count} of kernel."""
    cur = sqlite3.connect(db_path).cursor()
    gc = grid_column(cur)
    if not gc:
        return {}
    groups = {}
    for name, g in cur.execute(f"select name, {gc} from kernels"):
        if short_name(name).replace("mcpr::", "") == kernel:
            groups[int(g)] = groups.get(int(g), 0) + 1
    return groups


def counter_per_dispatch(db_path: str, kernel: str, grid=None):
    """Counter values of kernel's dispatches (grid: only those with that x
    extent in work items) and the largest value of a library copy."""
    cur = sqlite3.connect(db_path).cursor()
    q = list(cur.execute("select kernel_name, value, grid_size_x from counters_collection"))
    vals = [v for k, v, g in q if short_name(k).replace("mcpr::", "") == kernel and (grid is None or int(g) == grid)]
    copies = [v for k, v, g in q if "copyBuffer" in k]
    return vals, (max(copies) if copies else None)


def counters_of(db_path: str, kernel: str, grid=None):
    """Mean value per dispatch of every counter collected for kernel."""
    cur = sqlite3.connect(db_path).cursor()
    vals = {}
    for k, name, v, g in cur.execute("select kernel_name, counter_name, value, grid_size_x from counters_collection"):
        if short_name(k).replace("mcpr::", "") == kernel and (grid is None or int(g) == grid):
            vals.setdefault(name, []).append(v)
    return {n: (statistics.mean(v), len(v)) for n, v in vals.items()}


# MI355X: 256 compute units of 4 SIMDs; a wave64 VALU instruction occupies its
# SIMD for at least 4 cycles (16 lanes per cycle); 2.4 GHz peak engine clock.
SIMDS, VALU_CYCLES, CLOCK_HZ = 1024, 4, 2.4e9


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--kernel", default=None)
    t.add_argument("--grid", type=int, default=None, help="also the dispatches of --kernel with this grid x extent")
    t.add_argument("--bench-log", default=None)
    c = sub.add_parser("traffic")
    c.add_argument("fetch_db")
    c.add_argument("write_db")
    c.add_argument("--kernel", required=True)
    c.add_argument("--copy-mib", type=int, default=1024)
    c.add_argument("--algorithmic-bytes", type=float, required=True)
    c.add_argument("--grid", type=int, default=None, help="only dispatches with this grid x extent (work items)")
    v = sub.add_parser("valu")
    v.add_argument("db")
    v.add_argument("--kernel", required=True)
    v.add_argument("--trace-us", type=float, required=True, help="mean duration of the kernel (kernel trace)")
    v.add_argument("--grid", type=int, default=None, help="only dispatches with this grid x extent (work items)")
    a = ap.parse_args()
    if a.cmd == "trace":
        print("| kernel | calls | total us | mean us | % |")
        print("|---|---|---|---|---|")
        for name, calls, tot, avg, pct in kernel_table(a.db):
            print(f"| `{name}` | {calls} | {tot:.1f} | {avg:.2f} | {pct:.2f} |")
        if a.kernel:
            d = durations(a.db, a.kernel)
            if d:
                print(f"\n`{a.kernel}`: {len(d)} dispatches, mean {statistics.mean(d):.2f} us, median "
                      f"{statistics.median(d):.2f} us, min {min(d):.2f} us, max {max(d):.2f} us")
            groups = grid_groups(a.db, a.kernel)
            if len(groups) > 1 or a.grid:
                print("\n| grid (work items) | dispatches | mean us | median us |")
                print("|---|---|---|---|")
                for g in sorted(groups, reverse=True)[:8]:
                    dg = durations(a.db, a.kernel, g)
                    print(f"| {g} | {len(dg)} | {statistics.mean(dg):.2f} | {statistics.median(dg):.2f} |")
            if a.grid:
                dg = durations(a.db, a.kernel, a.grid)
                if dg:
                    print(f"\n`{a.kernel}` at grid {a.grid} (the launches of the timed steps' full sweeps): "
                          f"{len(dg)} dispatches, mean {statistics.mean(dg):.2f} us, median "
                          f"{statistics.median(dg):.2f} us")
        if a.bench_log:
            for line in open(a.bench_log):
                if line.startswith("{"):
                    r = json.loads(line)["roofline"]
                    print(f"\nbench.py, same run: {r['kernel']} mean {r['avg_launch_us']} us per launch by HIP events, "
                          f"{r['achieved']} GB/s algorithmic")
    elif a.cmd == "valu":
        cs = counters_of(a.db, a.kernel, a.grid)
        print("| counter | mean per dispatch | dispatches |")
        print("|---|---|---|")
        for name in sorted(cs):
            print(f"| {name} | {cs[name][0]:.6g} | {cs[name][1]} |")
        insts = cs["SQ_INSTS_VALU"][0]
        t_issue = insts * VALU_CYCLES / (SIMDS * CLOCK_HZ) * 1e6
        print(f"\nVALU issue time at full rate: {insts:.4g} wave instructions x {VALU_CYCLES} cycles / "
              f"({SIMDS} SIMDs x {CLOCK_HZ / 1e9:.1f} GHz) = {t_issue:.2f} us; kernel {a.trace_us:.2f} us; "
              f"ratio {t_issue / a.trace_us:.3f}")
        print(json.dumps({"valu_insts_per_launch": insts, "valu_issue_us": t_issue, "valu_frac": t_issue / a.trace_us}))
    else:
        kib = a.copy_mib * 1024.0
        out = {}
        for name, db in (("FETCH_SIZE", a.fetch_db), ("WRITE_SIZE", a.write_db)):
            vals, copy = counter_per_dispatch(db, a.kernel, a.grid)
            scale = kib / copy
            out[name] = dict(n=len(vals), raw_kib=statistics.mean(vals), copy_kib=copy, scale=scale,
                             bytes=statistics.mean(vals) * scale * 1024.0)
        tot = out["FETCH_SIZE"]["bytes"] + out["WRITE_SIZE"]["bytes"]
        print("| counter | copy of %d MiB reads (KiB) | scale | kernel raw KiB per dispatch | scaled bytes per dispatch |"
              % a.copy_mib)
        print("|---|---|---|---|---|")
        for name in ("FETCH_SIZE", "WRITE_SIZE"):
            o = out[name]
            print(f"| {name} | {o['copy_kib']:.0f} | {o['scale']:.4f} | {o['raw_kib']:.1f} ({o['n']} dispatches) | "
                  f"{o['bytes']:.4e} |")
        print(f"\ntraffic per dispatch {tot:.4e} B; algorithmic {a.algorithmic_bytes:.4e} B; "
              f"ratio {tot / a.algorithmic_bytes:.4f}")
        print(json.dumps({"bytes_per_launch": tot, "fetch_bytes": out["FETCH_SIZE"]["bytes"],
                          "write_bytes": out["WRITE_SIZE"]["bytes"]}))


if __name__ == "__main__":
    main()
