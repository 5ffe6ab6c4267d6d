"""Summaries of rocprofv3 result databases (SQLite, rocpd format) as short
Markdown tables.

    python -m paper_2008_00409_amd.profile_summary trace <results.db> [--top 15]
        per-kernel calls, mean / min / max duration and share of GPU time

    python -m paper_2008_00409_amd.profile_summary pmc <fetch.db> <write.db> --kernel NAME
            --copy-kernel NAME --copy-bytes N
        FETCH_SIZE and WRITE_SIZE per dispatch of one kernel (median over its
        full dispatches), scaled by what the same counters read for a plain
        copy kernel that moves N bytes each way; prints the scale factors and
        the HBM bytes per launch

    python -m paper_2008_00409_amd.profile_summary kernels <fetch.db> <write.db> <trace.db> [--sq <sq.db>]
            --kernel NAME [--kernel NAME ...] --copy-kernel NAME --copy-bytes N
        per kernel: mean duration, HBM bytes fetched and written per
        dispatch (copy-scaled as above), their rate, and with --sq the
        VALU instructions per wave

    python -m paper_2008_00409_amd.profile_summary counters <results.db> [...] --kernel NAME [--kernel NAME ...]
        every counter the databases hold, median over each kernel's
        dispatches (several databases: one counter pass each)
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sqlite3
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
# Sources the SpMV kernel is built from: a traffic figure stays valid only
# while they are unchanged.
SPMV_SOURCES = ["csrc/pc_spmv.h", "csrc/pc_common.h"]


def spmv_source_hash() -> str:
    h = hashlib.sha256()
    for rel in SPMV_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_rows(db):
    con = sqlite3.connect(db)
    return con.execute("select name, start, end, grid_x from kernels").fetchall()


def trace_table(db, top=15, by_grid=False):
    """Per-kernel table; with by_grid, launches of one kernel with different
    grid sizes (different workloads or schedules) are listed separately."""
    rows = kernel_rows(db)
    per = {}
    for name, s, e, gx in rows:
        key = (name, gx if by_grid else 0)
        per.setdefault(key, []).append((e - s) / 1e3)
    total = sum(sum(v) for v in per.values())
    head = "| kernel | grid threads | calls" if by_grid else "| kernel | calls"
    out = [head + " | mean us | mean us, full launches | min us | max us | share |",
           "|---|---|---|---|---|---|---|" + ("---|" if by_grid else "")]
    for (name, gx), v in sorted(per.items(), key=lambda kv: -sum(kv[1]))[:top]:
        short = name.split("(")[0].replace("void ", "")
        lead = f"| `{short}` | {gx} | {len(v)}" if by_grid else f"| `{short}` | {len(v)}"
        out.append(f"{lead} | {statistics.mean(v):.2f} | {full_mean(v):.2f} | {min(v):.2f} | "
                   f"{max(v):.2f} | {100 * sum(v) / total:.1f}% |")
    return "\n".join(out)


def counter_values(db, kernel_sub, counter):
    con = sqlite3.connect(db)
    q = "select kernel_name, dispatch_id, value from counters_collection where counter_name = ?"
    vals = {}
    for name, did, val in con.execute(q, (counter,)).fetchall():
        if kernel_sub in name:
            vals[did] = vals.get(did, 0.0) + val
    return list(vals.values())


def full_mean(vals):
    """Mean over launches that did the full work: CG launches after an
    instance has converged exit at once, so launches shorter than a quarter
    of the 90th percentile are left out."""
    p90 = sorted(vals)[int(0.9 * (len(vals) - 1))]
    full = [v for v in vals if v >= 0.25 * p90]
    return statistics.mean(full)


def full_median(vals):
    """Median over dispatches that did the full work (at least half of the
    largest value: launches that exit early after convergence are left out)."""
    if not vals:
        return float("nan")
    mx = max(vals)
    return statistics.median([v for v in vals if v >= 0.5 * mx])


def pmc_table(fetch_db, write_db, kernel, copy_kernel, copy_bytes):
    f_k = full_median(counter_values(fetch_db, kernel, "FETCH_SIZE"))
    w_k = full_median(counter_values(write_db, kernel, "WRITE_SIZE"))
    f_c = full_median(counter_values(fetch_db, copy_kernel, "FETCH_SIZE"))
    w_c = full_median(counter_values(write_db, copy_kernel, "WRITE_SIZE"))
    kib = copy_bytes / 1024.0
    sf, sw = kib / f_c, kib / w_c
    fetch = f_k * sf * 1024.0
    write = w_k * sw * 1024.0
    lines = [
        "| quantity | value |", "|---|---|",
        f"| copy kernel FETCH_SIZE (KiB / dispatch) | {f_c:.0f} (true {kib:.0f}: scale {sf:.3f}) |",
        f"| copy kernel WRITE_SIZE (KiB / dispatch) | {w_c:.0f} (true {kib:.0f}: scale {sw:.3f}) |",
        f"| `{kernel}` FETCH_SIZE (KiB / dispatch, raw) | {f_k:.0f} |",
        f"| `{kernel}` WRITE_SIZE (KiB / dispatch, raw) | {w_k:.0f} |",
        f"| `{kernel}` HBM bytes fetched / launch (scaled) | {fetch:.0f} |",
        f"| `{kernel}` HBM bytes written / launch (scaled) | {write:.0f} |",
        "",
        f"traffic_bytes_per_launch: {fetch + write:.0f}",
        f"kernel: {kernel}",
        f"spmv_source_hash: {spmv_source_hash()}",
    ]
    return "\n".join(lines)


def counter_names(db):
    con = sqlite3.connect(db)
    return [r[0] for r in con.execute("select distinct counter_name from counters_collection").fetchall()]


def counters_table(dbs, kernels):
    """One row per kernel, one column per counter: the median per dispatch."""
    cols, vals = [], {}
    for db in dbs:
        for cn in counter_names(db):
            cols.append(cn)
            for k in kernels:
                v = counter_values(db, k, cn)
                vals[(k, cn)] = statistics.median(v) if v else float("nan")
    out = ["| kernel | " + " | ".join(cols) + " |", "|---|" + "---|" * len(cols)]
    for k in kernels:
        out.append(f"| `{k}` | " + " | ".join(f"{vals[(k, c)]:.6g}" for c in cols) + " |")
    return "\n".join(out)


def kernels_table(fetch_db, write_db, trace_db, kernels, copy_kernel, copy_bytes, sq_db=None):
    kib = copy_bytes / 1024.0
    sf = kib / full_median(counter_values(fetch_db, copy_kernel, "FETCH_SIZE"))
    sw = kib / full_median(counter_values(write_db, copy_kernel, "WRITE_SIZE"))
    rows = kernel_rows(trace_db)
    out = [f"FETCH_SIZE scale {sf:.3f}, WRITE_SIZE scale {sw:.3f} (from `{copy_kernel}` moving {copy_bytes:.0f} B each way)",
           "",
           "| kernel | mean us | fetched MB | written MB | GB/s | VALU instructions per wave |",
           "|---|---|---|---|---|---|"]
    tb = tt = 0.0
    for k in kernels:
        f = statistics.median(counter_values(fetch_db, k, "FETCH_SIZE")) * sf * 1024.0
        w = statistics.median(counter_values(write_db, k, "WRITE_SIZE")) * sw * 1024.0
        t = statistics.mean([(e - s) / 1e3 for n, s, e, g in rows if k in n])
        va = "-"
        if sq_db:
            v = counter_values(sq_db, k, "SQ_INSTS_VALU")
            wv = counter_values(sq_db, k, "SQ_WAVES")
            if v and wv:
                va = f"{statistics.median(v) / statistics.median(wv):.0f}"
        tb += f + w
        tt += t
        out.append(f"| `{k}` | {t:.1f} | {f / 1e6:.1f} | {w / 1e6:.1f} | {(f + w) / (t * 1e-6) / 1e9:.0f} | {va} |")
    out.append(f"| all listed | {tt:.1f} | | {tb / 1e6:.1f} (total) | {tb / (tt * 1e-6) / 1e9:.0f} | |")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--top", type=int, default=15)
    t.add_argument("--by-grid", action="store_true")
    p = sub.add_parser("pmc")
    p.add_argument("fetch_db")
    p.add_argument("write_db")
    p.add_argument("--kernel", required=True)
    p.add_argument("--copy-kernel", required=True)
    p.add_argument("--copy-bytes", type=float, required=True)
    kk = sub.add_parser("kernels")
    kk.add_argument("fetch_db")
    kk.add_argument("write_db")
    kk.add_argument("trace_db")
    kk.add_argument("--sq", default=None)
    kk.add_argument("--kernel", action="append", required=True)
    kk.add_argument("--copy-kernel", required=True)
    kk.add_argument("--copy-bytes", type=float, required=True)
    c = sub.add_parser("counters")
    c.add_argument("dbs", nargs="+")
    c.add_argument("--kernel", action="append", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(trace_table(a.db, a.top, a.by_grid))
    elif a.cmd == "kernels":
        print(kernels_table(a.fetch_db, a.write_db, a.trace_db, a.kernel, a.copy_kernel, a.copy_bytes, a.sq))
    elif a.cmd == "counters":
        print(counters_table(a.dbs, a.kernel))
    else:
        print(pmc_table(a.fetch_db, a.write_db, a.kernel, a.copy_kernel, a.copy_bytes))


if __name__ == "__main__":
    main()
