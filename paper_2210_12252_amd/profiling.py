"""Summaries of rocprofv3 output databases (kernel durations, counters).

    python -m paper_2210_12252_amd.profiling stats  <results.db> [--title T] [--command C]
    python -m paper_2210_12252_amd.profiling counters <results.db> [--title T] [--command C]
    python -m paper_2210_12252_amd.profiling utilisation <results.db> [--kernels a,b] [--cus 256] [--title T]
    python -m paper_2210_12252_amd.profiling traffic --fetch <db> --write <db> --kernel K --name N
        --copy-bytes B --nvec V --hash H --workload W [--command C]

Prints a short markdown table: per kernel the dispatch count and the mean /
min / max duration in microseconds, and the mean over the later half of the
dispatches (``stats``), or the mean of every
collected counter per dispatch (``counters``).  Kernel names are shortened
to the function name and its template arguments.

``utilisation`` derives per-kernel rates from one counter run (means per
dispatch): kernel cycles = GRBM_GUI_ACTIVE / 8 (the counter sums the eight
XCDs; cycles at the shader clock), MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES /
(cycles x CUs x 4 SIMDs), VALU issue = 4 SQ_INSTS_VALU / (cycles x CUs x 4)
(a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles), MFMA work
= SQ_INSTS_VALU_MFMA_MOPS_* x 512 flops, LDS instructions and bank-conflict
cycles per CU and cycle, VALU and LDS activity as rocprofv3's own busy
metrics define them (SQ_ACTIVE_INST_* / (CUs x cycles)), and
SQ_WAIT_INST_ANY / SQ_BUSY_CU_CYCLES.

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
    """Per kernel: dispatches, mean / min / max / total duration (us) and the
    mean over the later half of its dispatches in launch order (with as many
    timed steps as warm-up steps, the timed steps of the bench command)."""
    c = sqlite3.connect(db)
    rows = c.execute("select name, count(*), avg(duration), min(duration), max(duration), sum(duration) "
                     "from kernels group by name order by sum(duration) desc").fetchall()
    out = []
    for n, cnt, avg, mn, mx, tot in rows:
        durs = [d for (d,) in c.execute("select duration from kernels where name = ? order by start", (n,))]
        late = durs[len(durs) // 2:]
        out.append((short_name(n), cnt, avg / 1e3, mn / 1e3, mx / 1e3, tot / 1e3, sum(late) / len(late) / 1e3))
    return out


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


def utilisation(db: str, kernels, cus: int, xcds: int = 8, clock_ghz: float = 2.4):
    """Derived rates per kernel (see the module docstring)."""
    per = {}
    for n, cn, v, k in counter_means(db):
        if kernels and not any(x in n for x in kernels):
            continue
        per.setdefault(n, {"dispatches": k})[cn] = v
    rows = []
    for n, c in per.items():
        cyc = c.get("GRBM_GUI_ACTIVE", 0.0) / xcds
        if cyc <= 0:
            continue
        simd = cyc * cus * 4
        r = {"kernel": n, "dispatches": c["dispatches"], "us": cyc / (clock_ghz * 1e3)}
        if "SQ_VALU_MFMA_BUSY_CYCLES" in c:
            r["mfma_busy"] = c["SQ_VALU_MFMA_BUSY_CYCLES"] / simd
        if "SQ_INSTS_VALU" in c:
            r["valu_issue"] = 4.0 * c["SQ_INSTS_VALU"] / simd
        mops = [(k, v) for k, v in c.items() if k.startswith("SQ_INSTS_VALU_MFMA_MOPS_")]
        if mops:
            r["mfma_tflops"] = sum(v for _, v in mops) * 512.0 / (r["us"] * 1e-6) / 1e12
            r["mfma_type"] = ",".join(k.rsplit("_", 1)[1] for k, _ in mops)
        if "SQ_ACTIVE_INST_VALU" in c:
            r["valu_active"] = c["SQ_ACTIVE_INST_VALU"] / (cyc * cus)
        if "SQ_ACTIVE_INST_LDS" in c:
            r["lds_active"] = c["SQ_ACTIVE_INST_LDS"] / (cyc * cus)
        if "SQ_INSTS_LDS" in c:
            r["lds_insts_per_cu_cycle"] = c["SQ_INSTS_LDS"] / (cyc * cus)
        if "SQ_LDS_BANK_CONFLICT" in c:
            r["lds_conflict_cycles_per_cu_cycle"] = c["SQ_LDS_BANK_CONFLICT"] / (cyc * cus)
        if "SQ_WAIT_INST_ANY" in c and c.get("SQ_BUSY_CU_CYCLES", 0) > 0:
            r["wait_any_per_busy_cu_cycle"] = c["SQ_WAIT_INST_ANY"] / c["SQ_BUSY_CU_CYCLES"]
        if "SQ_WAVES" in c:
            r["waves"] = c["SQ_WAVES"]
        r["raw"] = {k: v for k, v in c.items() if k != "dispatches"}
        rows.append(r)
    return rows


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
    ap.add_argument("mode", choices=("stats", "counters", "traffic", "utilisation"))
    ap.add_argument("--kernels", default="", help="utilisation: comma list of kernel-name substrings")
    ap.add_argument("--cus", type=int, default=256)
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
    if a.mode == "utilisation":
        ks = [k for k in a.kernels.split(",") if k]
        rows = utilisation(a.db, ks, a.cus)
        out.append("| kernel | dispatches | us | MFMA busy | MFMA TFLOP/s (type) | VALU issue | VALU active | LDS active "
                   "| LDS insts / CU-cycle | LDS conflict cycles / CU-cycle | SQ_WAIT_INST_ANY / SQ_BUSY_CU_CYCLES |")
        out.append("|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|")
        f = lambda r, k, fmt: (fmt % r[k]) if k in r else "-"   # noqa: E731
        for r in rows:
            mt = (f"{r['mfma_tflops']:.1f} ({r['mfma_type']})" if "mfma_tflops" in r else "-")
            out.append(f"| `{r['kernel']}` | {r['dispatches']} | {r['us']:.1f} | {f(r, 'mfma_busy', '%.3f')} | {mt} | "
                       f"{f(r, 'valu_issue', '%.3f')} | {f(r, 'valu_active', '%.3f')} | {f(r, 'lds_active', '%.3f')} | "
                       f"{f(r, 'lds_insts_per_cu_cycle', '%.4f')} | "
                       f"{f(r, 'lds_conflict_cycles_per_cu_cycle', '%.4f')} | "
                       f"{f(r, 'wait_any_per_busy_cu_cycle', '%.2f')} |")
        out.append("")
        out.append("Raw counters (mean per dispatch):")
        out.append("")
        for r in rows:
            out.append(f"- `{r['kernel']}`: " + ", ".join(f"{k} {v:.4g}" for k, v in sorted(r["raw"].items())))
    elif a.mode == "stats":
        out.append("| kernel | dispatches | mean us | mean us, later half | min us | max us | total us |")
        out.append("|---|---:|---:|---:|---:|---:|---:|")
        for n, cnt, avg, mn, mx, tot, late in kernel_stats(a.db):
            out.append(f"| `{n}` | {cnt} | {avg:.2f} | {late:.2f} | {mn:.2f} | {mx:.2f} | {tot:.1f} |")
    else:
        out.append("| kernel | counter | mean per dispatch | dispatches |")
        out.append("|---|---|---:|---:|")
        for n, cn, v, k in counter_means(a.db):
            out.append(f"| `{n}` | {cn} | {v:.1f} | {k} |")
    print("\n".join(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
