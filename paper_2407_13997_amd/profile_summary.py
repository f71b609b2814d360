"""Summarise rocprofv3 databases (rocpd SQLite) for the committed profiles.

  kernel-trace db:  per-kernel calls, total and average duration
  --pmc db:         per-kernel average of each counter per dispatch (FETCH_SIZE and
                    WRITE_SIZE in KiB, the SQ_ / GRBM_ counters in their own units)

With --by-grid the rows are split by launch grid size (work-items), so that
launches of one kernel on different workloads are reported apart.

Usage: python -m paper_2407_13997_amd.profile_summary [--by-grid] TRACE_DB [PMC_DB ...]
"""
from __future__ import annotations

import re
import sqlite3
import sys


def short(name: str) -> str:
    m = re.search(r"(k_\w+(<[^>(]*>)?|__amd\w+|at::native::\w+)", name)
    return m.group(0) if m else name[:60]


def kernel_stats(db: str, by_grid: bool):
    con = sqlite3.connect(db)
    grid, group = ("grid_x * grid_y * grid_z", "name, 2") if by_grid else ("0", "name")
    rows = con.execute(f"select name, {grid}, count(*), sum(end - start), avg(end - start), min(end - start), "
                       f"max(end - start) from kernels group by {group} "
                       "order by sum(end - start) desc").fetchall()
    return [(short(r[0]),) + tuple(r[1:]) for r in rows]


def pmc_stats(db: str, by_grid: bool):
    con = sqlite3.connect(db)
    grid, group = ("grid_size", "kernel_name, 2, counter_name") if by_grid else ("0", "kernel_name, counter_name")
    rows = con.execute(f"select kernel_name, {grid}, counter_name, count(*), avg(value), min(value), max(value) "
                       f"from counters_collection group by {group} "
                       "order by kernel_name").fetchall()
    return [(short(r[0]),) + tuple(r[1:]) for r in rows]


def main(argv):
    by_grid = "--by-grid" in argv
    argv = [a for a in argv if a != "--by-grid"]
    g_head, g_rule = ("grid | ", "---:|") if by_grid else ("", "")
    trace = argv[0]
    print(f"| kernel | {g_head}calls | total ms | avg ms | min ms | max ms |")
    print(f"|---|{g_rule}---:|---:|---:|---:|---:|")
    for n, gr, c, tot, avg, mn, mx in kernel_stats(trace, by_grid):
        g = f"{gr} | " if by_grid else ""
        print(f"| {n} | {g}{c} | {tot / 1e6:.3f} | {avg / 1e6:.4f} | {mn / 1e6:.4f} | {mx / 1e6:.4f} |")
    for db in argv[1:]:
        print()
        print(f"| kernel | {g_head}counter | dispatches | avg | min | max |")
        print(f"|---|{g_rule}---|---:|---:|---:|---:|")
        for n, gr, cn, c, avg, mn, mx in pmc_stats(db, by_grid):
            g = f"{gr} | " if by_grid else ""
            print(f"| {n} | {g}{cn} | {c} | {avg:.1f} | {mn:.1f} | {mx:.1f} |")


if __name__ == "__main__":
    main(sys.argv[1:])
