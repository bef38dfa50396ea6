"""Summaries of rocprofv3 output databases (kernel durations, counters).

    python -m paper_2210_12252_amd.profiling stats  <results.db> [--title T] [--command C]
    python -m paper_2210_12252_amd.profiling counters <results.db> [--title T] [--command C]

Prints a short markdown table: per kernel the dispatch count and the mean /
min / max duration in microseconds (``stats``), or the mean of every
collected counter per dispatch (``counters``).  Kernel names are shortened
to the function name and its template arguments.
"""
from __future__ import annotations

import argparse
import re
import sqlite3
import sys


def short_name(name: str) -> str:
    m = re.match(r"(?:void )?([\w:]+(?:<[^()]*>)?)\(", name)
    return m.group(1) if m else name[:80]


def kernel_stats(db: str):
    c = sqlite3.connect(db)
    rows = c.execute("select name, count(*), avg(duration), min(duration), max(duration), sum(duration) "
                     "from kernels group by name order by sum(duration) desc").fetchall()
    return [(short_name(n), cnt, avg / 1e3, mn / 1e3, mx / 1e3, tot / 1e3) for n, cnt, avg, mn, mx, tot in rows]


def counter_means(db: str):
    """Mean over dispatches of each counter, per kernel (a dispatch's rows,
    e.g. one per XCD or instance, are summed first)."""
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, counter_name, avg(s), count(*) from ("
                     "  select kernel_name, counter_name, dispatch_id, sum(value) as s from counters_collection"
                     "  group by kernel_name, counter_name, dispatch_id) "
                     "group by kernel_name, counter_name order by kernel_name, counter_name").fetchall()
    return [(short_name(n), cn, v, k) for n, cn, v, k in rows]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=("stats", "counters"))
    ap.add_argument("db")
    ap.add_argument("--title", default="")
    ap.add_argument("--command", default="")
    a = ap.parse_args(argv)
    out = []
    if a.title:
        out.append(f"# {a.title}\n")
    if a.command:
        out.append(f"Command: `{a.command}`\n")
    if a.mode == "stats":
        out.append("| kernel | dispatches | mean us | min us | max us | total us |")
        out.append("|---|---:|---:|---:|---:|---:|")
        for n, cnt, avg, mn, mx, tot in kernel_stats(a.db):
            out.append(f"| `{n}` | {cnt} | {avg:.2f} | {mn:.2f} | {mx:.2f} | {tot:.1f} |")
    else:
        out.append("| kernel | counter | mean per dispatch | dispatches |")
        out.append("|---|---|---:|---:|")
        for n, cn, v, k in counter_means(a.db):
            out.append(f"| `{n}` | {cn} | {v:.1f} | {k} |")
    print("\n".join(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
