"""Summaries of rocprofv3 output databases (kernel durations, counters).

    python -m paper_2210_12252_amd.profiling stats  <results.db> [--title T] [--command C]
    python -m paper_2210_12252_amd.profiling counters <results.db> [--title T] [--command C]
    python -m paper_2210_12252_amd.profiling traffic --fetch <db> --write <db> --kernel K --name N
        --copy-bytes B --nvec V --hash H --workload W [--command C]

Prints a short markdown table: per kernel the dispatch count and the mean /
min / max duration in microseconds (``stats``), or the mean of every
collected counter per dispatch (``counters``).  Kernel names are shortened
to the function name and its template arguments.

``traffic`` turns two counter runs of the same command (one collecting
FETCH_SIZE, one WRITE_SIZE; KiB per dispatch) into HBM bytes per launch of
the kernel whose name contains K (mean over its dispatches): each counter is
scaled by what it reads for the largest single dispatch of a plain device
copy in the run (B bytes read and B written),
and the result is printed as JSON (stage name, bytes per launch, the raw
counters, the scale factors, the kernel-source hash and the block size it
was taken at).
"""
from __future__ import annotations

import argparse
import re
import sqlite3
import sys


def short_name(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
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


def _counter_per_dispatch(db: str, counter: str):
    """{short kernel name: mean per dispatch} of one counter."""
    return {n: v for n, cn, v, _ in counter_means(db) if cn == counter}


def _counter_max(db: str, counter: str):
    """{short kernel name: largest per-dispatch value} of one counter."""
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, max(s) from ("
                     "  select kernel_name, dispatch_id, sum(value) as s from counters_collection"
                     "  where counter_name = ? group by kernel_name, dispatch_id) group by kernel_name",
                     (counter,)).fetchall()
    return {short_name(n): v for n, v in rows}


def traffic(a) -> dict:
    fetch = _counter_per_dispatch(a.fetch, "FETCH_SIZE")
    write = _counter_per_dispatch(a.write, "WRITE_SIZE")
    copies_f = {n: v for n, v in _counter_max(a.fetch, "FETCH_SIZE").items() if "copy" in n.lower()}
    copies_w = {n: v for n, v in _counter_max(a.write, "WRITE_SIZE").items() if "copy" in n.lower()}
    if not copies_f or not copies_w:
        raise SystemExit("no copy kernel in the counter runs (run the command with a copy probe)")
    cf = max(copies_f.values()) * 1024.0
    cw = max(copies_w.values()) * 1024.0
    rf, wf = a.copy_bytes / cf, a.copy_bytes / cw
    kf = [v for n, v in fetch.items() if a.kernel in n]
    kw = [v for n, v in write.items() if a.kernel in n]
    if not kf or not kw:
        raise SystemExit(f"kernel {a.kernel!r} not found in the counter runs")
    fb, wb = kf[0] * 1024.0 * rf, kw[0] * 1024.0 * wf
    return dict(name=a.name, kernel=a.kernel, workload=a.workload, bytes_per_launch=round(fb + wb), read_bytes=round(fb),
                write_bytes=round(wb), fetch_kib=kf[0], write_kib=kw[0], read_scale=round(rf, 4),
                write_scale=round(wf, 4), copy_bytes=a.copy_bytes, nvec=a.nvec, kernel_hash=a.hash,
                command=a.command)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=("stats", "counters", "traffic"))
    ap.add_argument("db", nargs="?")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--kernel")
    ap.add_argument("--name")
    ap.add_argument("--copy-bytes", type=float)
    ap.add_argument("--nvec", type=int)
    ap.add_argument("--hash")
    ap.add_argument("--workload")
    ap.add_argument("--title", default="")
    ap.add_argument("--command", default="")
    a = ap.parse_args(argv)
    if a.mode == "traffic":
        import json
        print(json.dumps(traffic(a), indent=1))
        return 0
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
