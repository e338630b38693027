"""Autotuner of the pair loops' cell-to-workgroup tiling.

The batched launch over cells of uneven occupancy has three knobs: the
sub-cell depth of the cell list (Morton order inside each cell, sub_bits),
the tile (ti particles per work item, k lanes per particle) and the
schedule (one workgroup per cell, or a work list taken by the hardware
grid, a static or a dynamic persistent grid). sph_autotune times every
(tile, schedule) candidate of one loop on a binned and converted particle
set; this driver repeats that for each sub-cell depth (which needs a
re-bin), picks the depth with the smallest density + force time and the
fastest candidate of each loop, and keeps the result in a JSON cache keyed
by the workload's signature (particle count, cells, occupancy statistics,
storage formats, device). On cells of very uneven occupancy it then tries
splitting each loop into two launches by an occupancy threshold T: the
cells with fewer than T particles with a tile of their own (optionally with
up to four such cells along x merged into one work item), the others with
the loop's tile, and keeps a split that is faster than the single launch.
Before that, the fastest few candidates of each loop (timed back to back on
their own) are timed again where the loop runs in a step, right after the
kernel that precedes it (bin, convert, density, force), and the fastest
there is kept: a schedule that partitions a resident grid statically can
lose several per cent in that position while leading in isolation.
The choice changes only timings: every candidate computes the same
interactions (merged items take a merged cell's positions relative to the
group's first cell, which changes FP32 rounding only).
"""
import json
import os

import numpy as np

from . import sphmi
from .pipeline import Pipeline

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "sphmi", "tune.json")


def signature(pipe: Pipeline) -> dict:
    """Workload signature of a binned pipeline: the tuner's cache key."""
    import torch
    start = pipe.cells.cell_start.cpu().numpy()
    occ = np.diff(start)
    p = pipe.prec
    props = torch.cuda.get_device_properties(pipe.aos.device)
    return {
        "abi": sphmi.abi_version(),
        "device": f"{props.gcnArchName.split(':')[0]}/{props.multi_processor_count}cu",
        "n": pipe.n, "n_c": pipe.n_c,
        "occ_max": int(occ.max()) if occ.size else 0,
        "occ_p50": float(np.median(occ)) if occ.size else 0.0,
        "occ_p99": float(np.percentile(occ, 99)) if occ.size else 0.0,
        "formats": [p.pos, p.vel, p.mhu, p.scale_m, p.scale_h, p.scale_u, p.pos_anchor],
    }


def _key(sig: dict) -> str:
    return json.dumps(sig, sort_keys=True)


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, cache):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


SPLIT_THRESHOLDS = (32, 48, 64)
# small-cell launches: (ti, k, sched, cells merged per work item at most)
SPLIT_SMALL = ((32, 2, "grid", 1), (32, 8, "grid", 1), (16, 4, "grid", 1), (64, 1, "grid", 1),
               (32, 2, "grid", 4), (64, 1, "grid", 4), (64, 2, "grid", 4))
SPLIT_LARGE = ((64, 4, "dynamic"), (32, 2, "grid"), (64, 4, "static"), (64, 1, "grid"))


def _small_str(sm) -> str:
    """'ti x k sched' of a small-cell launch, '+ merge m' when items merge cells."""
    out = f"{sm[0]}x{sm[1]} {sm[2]}"
    return out + (f" merge {sm[3]}" if len(sm) > 3 and sm[3] > 1 else "")


def _time_parts(pipe, loop, parts, reps):
    """Mean time (ms) of one pass of `loop` as the given launches."""
    import torch
    fn = sphmi.density if loop == "density" else sphmi.force

    def once():
        for til, w in parts:
            fn(pipe.soa, pipe.cells, pipe.prm, til, None, w)
    once()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        once()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_split(pipe, single: dict, reps: int = 3, log=None) -> dict:
    """For each loop, the best two-launch split (threshold T, small tile and
    schedule, large tile and schedule) on the binned and converted `pipe`,
    kept when it beats the single launch `single[loop]["ms"]` by 3 %."""
    occ = np.diff(pipe.cells.cell_start.cpu().numpy())
    out = {}
    works = {}

    def work(ti, sched, rng, merge=1):
        key = (ti, sched, rng, merge)
        if key not in works:
            w = sphmi.DeviceWork(pipe.n, pipe.n_c, ti, pipe.aos.device, sched, max_cells=merge)
            sphmi.worklist(pipe.cells, w, None, rng)
            works[key] = w
        return works[key]

    for loop in ("density", "force"):
        s = single[loop]
        large = {(s["ti"], s["k"], s["sched"] or "grid")} | set(SPLIT_LARGE)
        best = None
        for T in SPLIT_THRESHOLDS:
            frac = occ[occ < T].sum() / max(occ.sum(), 1)
            if not 0.05 < frac < 0.95:
                continue
            for (ts, ks, ss, ms_) in SPLIT_SMALL:
                for (tl, kl, sl) in sorted(large):
                    parts = [(sphmi.tile(ts, ks), work(ts, ss, (0, T), ms_)),
                             (sphmi.tile(tl, kl), work(tl, sl, (T, 2 ** 31 - 1)))]
                    ms = _time_parts(pipe, loop, parts, reps)
                    if best is None or ms < best[0]:
                        best = (ms, T, (ts, ks, ss, ms_), (tl, kl, sl))
        if best is not None and best[0] < 0.97 * s["ms"]:
            ms, T, sm, lg = best
            out[loop] = {"threshold": T, "small": list(sm), "large": list(lg), "ms": ms}
            if log:
                log(f"tune split {loop}: cells < {T} {_small_str(sm)}, others "
                    f"{lg[0]}x{lg[1]} {lg[2]}: {ms:.3f} ms (single {s['ms']:.3f} ms)")
    del works
    return out


REFINE_TOP = 3


def _in_step_ms(rec, n_c, prec, prm, sb, d, f, reps):
    """Mean density and force times (ms) inside the sequence bin, convert,
    density, force, for the tiles d and f = (ti, k, sched)."""
    import torch
    pipe = Pipeline(rec, n_c, prec=prec, prm=prm, sub_bits=sb, til=sphmi.tile(d[0], d[1]),
                    til_force=sphmi.tile(f[0], f[1]), sched=(d[2], f[2]))
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps + 1)]
    for r in range(reps + 1):               # the first pass is a warmup
        pipe.bin()
        pipe.convert("full")
        ev[r][0].record()
        pipe.density()
        ev[r][1].record()
        pipe.force()
        ev[r][2].record()
    torch.cuda.synchronize()
    dm = sum(ev[r][0].elapsed_time(ev[r][1]) for r in range(1, reps + 1)) / reps
    fm = sum(ev[r][1].elapsed_time(ev[r][2]) for r in range(1, reps + 1)) / reps
    del pipe
    return dm, fm


def refine_in_step(rec, n_c, prec, prm, sb, table, choice, reps=4, log=None):
    """Re-times the REFINE_TOP fastest isolated candidates of each loop (at
    sub-cell depth sb) in their place in a step and returns {loop: (ti, k,
    sched, ms)} of the fastest there."""
    import torch
    out = {}
    for loop in ("density", "force"):
        rows = sorted((r for r in table if r["sub_bits"] == sb and r["loop"] == loop),
                      key=lambda r: r["ms"])
        cands = []
        for r in rows:
            c = (r["ti"], r["k"], r["sched"])
            if c not in cands:
                cands.append(c)
            if len(cands) == REFINE_TOP:
                break
        best = None
        for c in cands:
            d = c if loop == "density" else choice["density"]
            f = c if loop == "force" else choice["force"]
            ms = _in_step_ms(rec, n_c, prec, prm, sb, d, f, reps)[0 if loop == "density" else 1]
            if log:
                log(f"tune in step {loop}: {c[0]}x{c[1]} {c[2] or 'per-cell'} {ms:.3f} ms")
            if best is None or ms < best[3]:
                best = (c[0], c[1], c[2], ms)
        out[loop] = best
        torch.cuda.empty_cache()
    return out


def tune(rec: np.ndarray, n_c: int, prec=None, prm=None, sub_bits=(0, 1, 2), cand=None,
         reps: int = 3, cache_path=DEFAULT_CACHE, refresh: bool = False, log=None,
         split: bool = True, refine: bool = True) -> dict:
    """Choose sub_bits and each loop's (tile, schedule) for the AoS records
    `rec` binned with n_c cells per axis. Returns {"sub_bits", "density":
    {ti, k, sched, ms}, "force": {...}, "table": [...], "signature", "cached"}."""
    import torch
    first = Pipeline(rec, n_c, prec=prec, prm=prm, sub_bits=sub_bits[0])
    first.bin()
    sig = signature(first)
    sig["sub_bits"] = list(sub_bits)
    sig["reps"] = reps
    sig["candidates"] = cand if cand is None else [list(c) for c in cand]
    sig["split"] = bool(split)
    sig["refine"] = bool(refine)
    cache = _load(cache_path) if cache_path else {}
    if not refresh and _key(sig) in cache:
        out = dict(cache[_key(sig)])
        out["cached"] = True
        return out
    cand = cand if cand is not None else sphmi.tune_candidates()
    tis = sorted({c[0] for c in cand})
    wbytes = max(sphmi.worklist_size(first.n, n_c, t) for t in tis)
    wbuf = torch.empty(wbytes, dtype=torch.uint8, device=first.aos.device)
    table, best = [], None
    for sb in sub_bits:
        pipe = first if sb == sub_bits[0] else Pipeline(rec, n_c, prec=prec, prm=prm, sub_bits=sb)
        pipe.bin()
        pipe.convert("full")
        dres, di = sphmi.autotune("density", pipe.soa, pipe.cells, pipe.prm, cand, reps, wbuf)
        fres, fi = sphmi.autotune("force", pipe.soa, pipe.cells, pipe.prm, cand, reps, wbuf)
        for loop, res in (("density", dres), ("force", fres)):
            table += [{"sub_bits": sb, "loop": loop, "ti": t, "k": k, "sched": s, "ms": ms}
                      for (t, k, s, ms) in res]
        d, f = dres[di], fres[fi]
        tot = d[3] + f[3]
        if log:
            log(f"tune sub_bits={sb}: density {d[0]}x{d[1]} {d[2]} {d[3]:.3f} ms, "
                f"force {f[0]}x{f[1]} {f[2]} {f[3]:.3f} ms")
        if best is None or tot < best[0]:
            best = (tot, sb, d, f)
        if pipe is not first:
            del pipe
    del first, wbuf
    torch.cuda.empty_cache()
    _, sb, d, f = best
    if refine:
        rf = refine_in_step(rec, n_c, prec, prm, sb, table,
                            {"density": (d[0], d[1], d[2]), "force": (f[0], f[1], f[2])},
                            log=log)
        # the isolated times of the kept candidates (the split search compares
        # against isolated launches)
        iso = {(r["loop"], r["ti"], r["k"], r["sched"]): r["ms"] for r in table if r["sub_bits"] == sb}
        d = rf["density"][:3] + (iso[("density",) + rf["density"][:3]],)
        f = rf["force"][:3] + (iso[("force",) + rf["force"][:3]],)
    out = {"sub_bits": sb,
           "density": {"ti": d[0], "k": d[1], "sched": d[2], "ms": d[3]},
           "force": {"ti": f[0], "k": f[1], "sched": f[2], "ms": f[3]},
           "table": table, "signature": sig, "split": {}}
    if split:
        pipe = Pipeline(rec, n_c, prec=prec, prm=prm, sub_bits=sb)
        pipe.bin()
        pipe.convert("full")
        out["split"] = tune_split(pipe, out, reps, log)
        del pipe
        torch.cuda.empty_cache()
    if cache_path:
        cache = _load(cache_path)
        cache[_key(sig)] = out
        _store(cache_path, cache)
    out = dict(out)
    out["cached"] = False
    return out


def pipeline_kwargs(choice: dict) -> dict:
    """Pipeline keyword arguments that apply a tuner choice."""
    d, f = dict(choice["density"]), dict(choice["force"])
    sp = choice.get("split") or {}
    split = {}
    for loop, c in (("density", d), ("force", f)):
        if loop in sp:
            s = sp[loop]
            c["ti"], c["k"], c["sched"] = s["large"]
            sm = list(s["small"]) + [1] * (4 - len(s["small"]))
            split[loop] = (s["threshold"], (sm[0], sm[1]), sm[2], sm[3])
    return {"sub_bits": choice["sub_bits"], "til": sphmi.tile(d["ti"], d["k"]),
            "til_force": sphmi.tile(f["ti"], f["k"]), "sched": (d["sched"], f["sched"]),
            "split": split}


def describe(choice: dict) -> str:
    out = [f"sub_bits {choice['sub_bits']}"]
    sp = choice.get("split") or {}
    for loop in ("density", "force"):
        if loop in sp:
            s = sp[loop]
            out.append(f"{loop} cells < {s['threshold']}: {_small_str(s['small'])}, "
                       f"others {s['large'][0]}x{s['large'][1]} {s['large'][2]}")
        else:
            c = choice[loop]
            out.append(f"{loop} {c['ti']}x{c['k']} {c['sched'] or 'per-cell'}")
    return "; ".join(out)
