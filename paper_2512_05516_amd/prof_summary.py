"""Summarise rocprofv3 databases of a bench run into a short text table.

    python -m paper_2512_05516_amd.prof_summary KTRACE.db [--fetch FETCH.db]
        [--write WRITE.db] [--copy-bytes N] [--title T]
        [--traffic-kernel SUBSTR --tiling T] [--pmc DB ... --pmc-kernel SUBSTR]

Kernel trace: calls and average / min / max duration per kernel. Counter
runs (FETCH_SIZE, WRITE_SIZE in KiB per dispatch): the per-kernel average,
and, when --copy-bytes is given, the factor that makes the counters of the
largest device copy (the library's k_probe_copy) read its known size,
applied to every kernel. --traffic-kernel adds one machine-readable line with the
scaled FETCH + WRITE bytes per launch of that kernel, the tiling the run
used and the SHA-256 of the kernel's sources (source_hash()), so a reader
can tell whether the counters still describe the current code. --pmc lists
counter databases of other runs (SQ_* instruction and cycle counters): for
every kernel whose name contains a --pmc-kernel substring, the average per
dispatch of each counter, and derived figures: VALU lane-instructions per
in-support pair when --pairs gives kernel=pairs (per launch), and the VALU
issue rate SQ_INSTS_VALU / (GRBM_GUI_ACTIVE / 8 XCDs x 256 CUs).
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sqlite3
import sys
from collections import defaultdict

# sources of the FP32 SoA pair kernels (the dominant kernel of the step)
KERNEL_SOURCES = ("csrc/pair_impl.h", "csrc/pair_force_f32.hip", "csrc/pair_dens_f32.hip",
                  "csrc/sph_device.h")


def source_hash() -> str:
    here = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(here, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def read_traffic(path: str):
    """The first traffic line of a summary file as a dict, or None."""
    lines = read_traffic_all(path)
    return lines[0] if lines else None


def read_traffic_all(path: str):
    """Every traffic line of a summary file (one per profiled kernel
    instance) as a list of dicts; empty if the file is missing."""
    out = []
    try:
        with open(path) as fh:
            for line in fh:
                if line.startswith("traffic "):
                    out.append(dict(kv.split("=", 1) for kv in line.split()[1:]))
    except OSError:
        pass
    return out


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
        if "k_probe_copy" in name:
            copies.append((grid, val))
    return agg, copies


def counter_table(dbs, substrs):
    """{kernel: {counter: average per dispatch}} over the databases, for the
    kernels whose (short) name contains one of substrs."""
    out = defaultdict(dict)
    for db in dbs:
        cur = sqlite3.connect(db).cursor()
        rows = cur.execute("select kernel_name, counter_name, value from counters_collection"
                           ).fetchall()
        agg = defaultdict(list)
        for name, cname, val in rows:
            sn = short(name)
            if any(x in sn for x in substrs):
                agg[(sn, cname)].append(val)
        for (sn, cname), v in agg.items():
            out[sn][cname] = sum(v) / len(v)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("ktrace")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-bytes", type=int, default=0)
    ap.add_argument("--title", default="")
    ap.add_argument("--traffic-kernel", default="")
    ap.add_argument("--tiling", default="")
    ap.add_argument("--pmc", nargs="*", default=[])
    ap.add_argument("--pmc-kernel", nargs="*", default=["k_force", "k_density"])
    ap.add_argument("--pairs", nargs="*", default=[],
                    help="SUBSTR=N: in-support pairs per launch of the kernels matching SUBSTR")
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
    per_launch = {}
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
            if a.traffic_kernel and a.traffic_kernel in name:
                per_launch[counter] = avg * scale * 1024.0
    if a.pmc:
        pairs = dict(kv.rsplit("=", 1) for kv in a.pairs)
        out.append("")
        out.append("counters per dispatch (average), " + " + ".join(os.path.basename(p) for p in a.pmc))
        for name, cnt in sorted(counter_table(a.pmc, a.pmc_kernel).items()):
            out.append(f"{name}:")
            out.append("    " + ", ".join(f"{c} {v:.4g}" for c, v in sorted(cnt.items())))
            extra = []
            if "SQ_INSTS_VALU" in cnt and "GRBM_GUI_ACTIVE" in cnt and cnt["GRBM_GUI_ACTIVE"] > 0:
                cyc = cnt["GRBM_GUI_ACTIVE"] / 8.0
                extra.append(f"{cyc:.3g} cycles per XCD; VALU issue "
                             f"{100 * cnt['SQ_INSTS_VALU'] / (cyc * 256):.1f}%")
            for sub, npairs in pairs.items():
                if sub in name and "SQ_INSTS_VALU" in cnt:
                    extra.append(f"{64 * cnt['SQ_INSTS_VALU'] / float(npairs):.0f} VALU "
                                 f"lane-instructions per pair")
                    f32 = [cnt.get(f"SQ_INSTS_VALU_{k}_F32") for k in ("FMA", "MUL", "ADD", "TRANS")]
                    if all(v is not None for v in f32):
                        flop = 64 * (2 * f32[0] + f32[1] + f32[2] + f32[3]) / float(npairs)
                        extra.append(f"{flop:.0f} FP32 flop per pair executed (FMA = 2)")
            if extra:
                out.append("    -> " + "; ".join(extra))
    if a.traffic_kernel and len(per_launch) == 2:
        out.append("")
        out.append(f"traffic kernel={a.traffic_kernel.replace(' ', '')} tiling={a.tiling} "
                   f"fetch_bytes={per_launch['FETCH_SIZE']:.0f} "
                   f"write_bytes={per_launch['WRITE_SIZE']:.0f} source_sha256={source_hash()}")
    print("\n".join(out))


if __name__ == "__main__":
    sys.exit(main())
