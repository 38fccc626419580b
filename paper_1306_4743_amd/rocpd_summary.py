"""Summarise a rocprofv3 results database (rocpd SQLite) as short text.

Usage: python -m paper_1306_4743_amd.rocpd_summary <results.db> [--pmc] [--match TEXT ...]

Prints per-kernel call counts and durations (total, average, min, max) and, with --pmc, the
average of every collected counter per dispatch of each kernel.  Only the standard library is
used, so it runs where the database was copied to, without a GPU.
"""
from __future__ import annotations

import argparse
import sqlite3
import statistics


def kernel_table(con, match=None):
    rows = con.execute("select name, duration from kernels").fetchall()
    by = {}
    for name, dur in rows:
        if match and not any(m in name for m in match):
            continue
        by.setdefault(name, []).append(float(dur))
    out = []
    for name, ds in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        out.append((name, len(ds), sum(ds) / 1e6, statistics.mean(ds) / 1e6, min(ds) / 1e6,
                    max(ds) / 1e6))
    return out


def pmc_table(con):
    try:
        rows = con.execute("select * from counters_collection").fetchall()
        cols = [r[1] for r in con.execute("pragma table_info(counters_collection)")]
    except sqlite3.OperationalError:
        return []
    ci = {c: i for i, c in enumerate(cols)}
    name_col = "kernel_name" if "kernel_name" in ci else "name"
    acc = {}
    for r in rows:
        key = (r[ci[name_col]], r[ci["counter_name"]])
        acc.setdefault(key, {}).setdefault(r[ci["dispatch_id"]], 0.0)
        acc[key][r[ci["dispatch_id"]]] += float(r[ci["value"]])
    out = []
    for (kname, cname), per in sorted(acc.items()):
        vals = list(per.values())
        out.append((kname, cname, len(vals), statistics.mean(vals)))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--pmc", action="store_true")
    ap.add_argument("--match", action="append",
                    help="only kernels whose name contains this text (repeatable)")
    a = ap.parse_args()
    con = sqlite3.connect(a.db)
    print("| kernel | calls | total ms | avg ms | min ms | max ms |")
    print("|---|---|---|---|---|---|")
    for name, n, tot, avg, mn, mx in kernel_table(con, a.match):
        print(f"| `{name}` | {n} | {tot:.3f} | {avg:.3f} | {mn:.3f} | {mx:.3f} |")
    if a.pmc:
        print()
        print("| kernel | counter | dispatches | mean per dispatch |")
        print("|---|---|---|---|")
        for kname, cname, n, mean in pmc_table(con):
            print(f"| `{kname}` | {cname} | {n} | {mean:.1f} |")


if __name__ == "__main__":
    main()
