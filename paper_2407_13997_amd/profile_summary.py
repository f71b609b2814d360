"""Summarise rocprofv3 databases (rocpd SQLite) for the committed profiles.

  kernel-trace db:  per-kernel calls, total and average duration
  --pmc db:         per-kernel average of each counter per dispatch (FETCH_SIZE and
                    WRITE_SIZE in KiB, the SQ_ / GRBM_ counters in their own units)

Usage: python -m paper_2407_13997_amd.profile_summary TRACE_DB [PMC_DB ...]
"""
from __future__ import annotations

import re
import sqlite3
import sys


def short(name: str) -> str:
    m = re.search(r"(k_\w+(<[^>(]*>)?|__amd\w+|at::native::\w+)", name)
    return m.group(0) if m else name[:60]


def kernel_stats(db: str):
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), sum(end - start), avg(end - start), min(end - start), "
                       "max(end - start) from kernels group by name order by sum(end - start) desc").fetchall()
    return [(short(r[0]), r[1], r[2], r[3], r[4], r[5]) for r in rows]


def pmc_stats(db: str):
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, counter_name, count(*), avg(value), min(value), max(value) "
                       "from counters_collection group by kernel_name, counter_name "
                       "order by kernel_name").fetchall()
    return [(short(r[0]), r[1], r[2], r[3], r[4], r[5]) for r in rows]


def main(argv):
    trace = argv[0]
    print("| kernel | calls | total ms | avg ms | min ms | max ms |")
    print("|---|---:|---:|---:|---:|---:|")
    for n, c, tot, avg, mn, mx in kernel_stats(trace):
        print(f"| {n} | {c} | {tot / 1e6:.3f} | {avg / 1e6:.4f} | {mn / 1e6:.4f} | {mx / 1e6:.4f} |")
    for db in argv[1:]:
        print()
        print("| kernel | counter | dispatches | avg | min | max |")
        print("|---|---|---:|---:|---:|---:|")
        for n, cn, c, avg, mn, mx in pmc_stats(db):
            print(f"| {n} | {cn} | {c} | {avg:.1f} | {mn:.1f} | {mx:.1f} |")


if __name__ == "__main__":
    main(sys.argv[1:])
