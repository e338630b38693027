"""Summarise rocprofv3 databases of a bench run into a short text table.

    python -m paper_2512_05516_amd.prof_summary KTRACE.db [--fetch FETCH.db]
        [--write WRITE.db] [--copy-bytes N] [--title T]

Kernel trace: calls and average / min / max duration per kernel. Counter
runs (FETCH_SIZE, WRITE_SIZE in KiB per dispatch): the per-kernel average,
and, when --copy-bytes is given, the factor that makes the counters of the
largest device copy (__amd_rocclr_copyBuffer) read its known size, applied
to every kernel.
"""
from __future__ import annotations

import argparse
import sqlite3
import sys
from collections import defaultdict


def short(name: str) -> str:
    n = name.replace("sph::(anonymous namespace)::", "").replace("(anonymous namespace)::", "")
    if "(" in n and not n.startswith("void at::"):
        n = n[: n.index("(")]
    if n.startswith("void "):
        n = n[5:]
    return n[:90]


def kernel_stats(db):
    cur = sqlite3.connect(db).cursor()
    rows = cur.execute("select name, start, end from kernels").fetchall()
    agg = defaultdict(list)
    for name, s, e in rows:
        agg[short(name)].append((e - s) * 1e-3)
    return agg


def counter_avgs(db, counter):
    cur = sqlite3.connect(db).cursor()
    rows = cur.execute("select kernel_name, grid_size, value from counters_collection "
                       "where counter_name = ?", (counter,)).fetchall()
    agg = defaultdict(list)
    copies = []
    for name, grid, val in rows:
        agg[short(name)].append(val)
        if "copyBuffer" in name:
            copies.append((grid, val))
    return agg, copies


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("ktrace")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-bytes", type=int, default=0)
    ap.add_argument("--title", default="")
    a = ap.parse_args(argv)
    out = []
    if a.title:
        out.append(a.title)
    k = kernel_stats(a.ktrace)
    tot = sum(sum(v) for v in k.values())
    out.append(f"{'kernel':90s} {'calls':>5s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'pct':>6s}")
    for name, v in sorted(k.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"{name:90s} {len(v):5d} {sum(v)/len(v):9.1f} {min(v):9.1f} {max(v):9.1f} "
                   f"{100*sum(v)/tot:6.2f}")
    for counter, path in (("FETCH_SIZE", a.fetch), ("WRITE_SIZE", a.write)):
        if not path:
            continue
        agg, copies = counter_avgs(path, counter)
        scale = 1.0
        note = "raw"
        if a.copy_bytes and copies:
            big = max(copies)[1]
            scale = (a.copy_bytes / 1024.0) / big if big else 1.0
            note = (f"scaled by {scale:.4f} (copy of {a.copy_bytes} B read {big:.0f} KiB)")
        out.append("")
        out.append(f"{counter} per dispatch, KiB, {note}")
        for name, v in sorted(agg.items(), key=lambda kv: -sum(kv[1]) / len(kv[1])):
            avg = sum(v) / len(v)
            out.append(f"{name:90s} {len(v):5d} {avg * scale:14.1f}")
    print("\n".join(out))


if __name__ == "__main__":
    sys.exit(main())
