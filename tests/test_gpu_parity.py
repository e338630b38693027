"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: bit-exact for binning, permutation, cell starts and quantised storage
values; neighbour counts equal to the FP64 brute-force counts for every
particle with no pair within FP32 rounding of a support radius (the others
differ by at most their number of such pairs; they are a small fraction);
FP32 storage within 1e-5 relative of the FP64 oracle (rho, wcount,
f, P, c: max per-particle relative error; a, du/dt: relative RMSE normalised
by the mean magnitude as in the paper's Sec. 7, with the maximum normalised
error also bounded); reduced storage: kernel arithmetic checked against the
oracle on the same dequantised inputs (FP32 bar), and the storage error
against FP64 gated at 2e-3 (FP16: rho, a) and 8e-3 (BF16 velocities:
du/dt).
"""
import numpy as np
import pytest

from paper_2512_05516_amd import inputs

from helpers import (assert_counts, brick_order, gpu_fields, max_rel, oracle_step, rel_max,
                     rel_rmse, run_gpu, unpack_trunc)

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5


@pytest.fixture(scope="module")
def sph():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_05516_amd import sphmi
    sphmi.lib()          # raises if the HIP library is missing: no fallback
    return sphmi


def check_fp32(got, d, f, tol=FP32_TOL, tag=""):
    errs = {
        "rho": max_rel(got["rho"], d["rho"]),
        "wcount": max_rel(got["wcount"], d["wcount"]),
        "f": max_rel(got["f"], d["f"]),
        "P": max_rel(got["P"], d["P"]),
        "c": max_rel(got["c"], d["c"]),
        # rho_dh enters only through h/(3 rho) rho_dh (the grad-h term)
        "omega": float(np.max(np.abs((got["rho_dh"] - d["rho_dh"]) * got["h"] / (3 * d["rho"])))),
        "a_rmse": rel_rmse(got["a"], f["a"]),
        "du_rmse": rel_rmse(got["du"], f["du"]),
        "vsig": max_rel(got["vsig"], f["vsig"]),
    }
    print(tag, {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= tol, (tag, k, v)
    assert rel_max(got["a"], f["a"]) <= 20 * tol, tag
    assert rel_max(got["du"], f["du"]) <= 20 * tol, tag
    return errs


# ---------------------------------------------------------------------------
# binning
# ---------------------------------------------------------------------------

def _bin_gpu(sph, x, n_c, sub_bits=0, h=None):
    import torch
    from paper_2512_05516_amd.pipeline import Pipeline
    hh = np.ones(len(x)) if h is None else h
    ps = inputs.ParticleSet(x, np.zeros_like(x), np.ones(len(x)), hh, np.ones(len(x)))
    pipe = Pipeline(inputs.pack_aos(ps, "f32"), n_c, sub_bits=sub_bits)
    pipe.bin()
    torch.cuda.synchronize()
    n = len(x)
    out = (pipe.cells.cell_start.cpu().numpy(), pipe.cells.perm[:n].cpu().numpy(),
           pipe.cells.cell[:n].cpu().numpy(), pipe.status())
    if sub_bits or h is not None:
        sub = pipe.cells.sub_start.cpu().numpy() if sub_bits else None
        return out + (sub, pipe.cells.hmax.cpu().numpy())
    return out


# cell ids of 5 to 19 bits: one, two and three radix passes, 8- and 9-bit digits
@pytest.mark.parametrize("n,n_c", [(0, 3), (1, 3), (4096, 4), (20000, 7), (100003, 23),
                                    (150001, 50), (300000, 70)])
def test_bin_bit_exact(sph, orc, n, n_c):
    rng = np.random.default_rng(n + n_c)
    x = rng.uniform(-0.5, 1.5, size=(n, 3))
    if n >= 8:
        x[:8] = [[0, 0, 0], [1 - 1e-17, 0.5, 0.5], [-1e-18, 1 / 3, 2 / 3], [1.0, 1.0, 1.0],
                 [0.5, 0.25, 0.75], [1 / n_c, 2 / n_c, 3 / n_c], [-1.0, 2.0, 0.999999999],
                 [0.1, 0.2, 0.3]]
    start, perm, cell, status = _bin_gpu(sph, x, n_c)
    ocell, ostart, operm, _ = orc.bin_cells(x, n_c)
    assert status == 0
    assert np.array_equal(start, ostart)
    assert np.array_equal(perm, operm)
    assert np.array_equal(cell, ocell[operm])


# keys of 8 to 25 bits, including 9-bit digits in one, two and three passes
@pytest.mark.parametrize("n,n_c,bits", [(4096, 4, 1), (30011, 7, 2), (200000, 23, 3),
                                         (200000, 32, 1), (300000, 70, 2), (1, 3, 2), (0, 3, 1)])
def test_bin_sub_cells_bit_exact(sph, orc, n, n_c, bits):
    rng = np.random.default_rng(n + 7 * bits)
    x = rng.uniform(-0.5, 1.5, size=(n, 3))
    h = rng.uniform(0.01, 0.02, size=n)
    start, perm, cell, status, sub, hmax = _bin_gpu(sph, x, n_c, bits, h)
    key, osub, operm = orc.bin_sub(x, n_c, bits)
    ocell, ostart, _, _ = orc.bin_cells(x, n_c)
    assert status == 0
    assert np.array_equal(perm, operm)
    assert np.array_equal(sub, osub)
    assert np.array_equal(start, ostart)
    assert np.array_equal(cell, ocell[operm])
    # hmax: the largest stored (FP32) h of each cell, 0 for empty cells
    h32 = h.astype(np.float32)
    want = np.zeros(n_c ** 3, np.float32)
    np.maximum.at(want, ocell, h32)
    assert np.array_equal(hmax, want)


def test_bin_flags_non_finite(sph):
    x = np.random.default_rng(0).uniform(0, 1, size=(100, 3))
    x[5, 1] = np.nan
    x[7, 2] = np.inf
    start, perm, cell, status = _bin_gpu(sph, x, 3)
    assert status & sph.FLAG_BAD_POSITION
    assert start[-1] == 100 and sorted(perm.tolist()) == list(range(100))


# ---------------------------------------------------------------------------
# conversion (U o N o C) and storage formats
# ---------------------------------------------------------------------------

# (pos, vel, mhu, scales, position anchor: 0 corner, 1 + b sub-cell centre)
PRECS = [("f32", "f32", "f32", (0, 0, 0), 0), ("f16", "bf16", "f16", (12, 3, 0), 3),
         ("bf16", "f16", "bf16", (0, 0, 0), 0), ("f16", "f16", "f16", (21, 6, -1), 2),
         ("f32", "f16", "f32", (0, 0, 0), 1), ("f16", "bf16", "f16", (12, 3, 0), 0)]


@pytest.mark.parametrize("kind", ["f32", "f64"])
@pytest.mark.parametrize("pos,vel,mhu,scales,anchor", PRECS)
def test_convert_bit_exact(sph, orc, kind, pos, vel, mhu, scales, anchor):
    import torch
    from paper_2512_05516_amd.pipeline import Pipeline
    ps = inputs.small_set(3)
    ps.v = ps.v * 37.0            # spread of exponents in the velocity format
    n_c = 4
    rec = inputs.pack_aos(ps, kind)
    src = inputs.unpack_aos(rec)  # the values the record holds, FP64
    prec = sph.precision(pos, vel, mhu, *scales, anchor=anchor)
    pipe = Pipeline(rec, n_c, prec=prec)
    pipe.bin()
    pipe.convert("full")
    torch.cuda.synchronize()
    ocell, ostart, operm, _ = orc.bin_cells(src.x, n_c)
    off, code = orc.pos_offsets(src.x, n_c, anchor)
    if anchor >= 2:
        assert np.array_equal(pipe.soa["ANC"].cpu().numpy(), code[operm])

    def bits(t):
        t = t.cpu()
        return t.view(torch.int16).numpy().view(np.uint16) if t.element_size() == 2 else \
            t.view(torch.int32).numpy().view(np.uint32)

    def want_bits(vals64, fmt, scale=0):
        v32 = np.array([orc.roundtrip(float(v), "f32") for v in vals64], np.float32) * \
            np.float32(2.0 ** scale)
        return v32.view(np.uint32) if fmt == "f32" else orc.quant(v32, fmt)

    for a, name in enumerate(("OFF_X", "OFF_Y", "OFF_Z")):
        assert np.array_equal(bits(pipe.soa[name]), want_bits(off[operm, a], pos)), name
    for a, name in enumerate(("VQ_X", "VQ_Y", "VQ_Z")):
        assert np.array_equal(bits(pipe.soa[name]), want_bits(src.v[operm, a], vel)), name
    for name, vals, s in (("M", src.m, scales[0]), ("H", src.h, scales[1]), ("U", src.u, scales[2])):
        assert np.array_equal(bits(pipe.soa[name]), want_bits(vals[operm], mhu, s)), name
    xw = src.x - np.floor(src.x)
    for a, name in enumerate(("X_X", "X_Y", "X_Z")):
        assert np.array_equal(pipe.soa[name].cpu().numpy(), xw[operm, a])
    for a, name in enumerate(("V_X", "V_Y", "V_Z")):
        assert np.array_equal(pipe.soa[name].cpu().numpy(), src.v[operm, a].astype(np.float32))


@pytest.mark.parametrize("kind", ["lattice", "clustered"])
def test_host_convert_matches_device(sph, kind):
    """Host-side binning + gather gives the device's cell list (hmax
    included) and SoA bit for bit, and the pair loops after it agree bit
    for bit with the loops after the device convert."""
    import torch
    from paper_2512_05516_amd.pipeline import Pipeline
    if kind == "lattice":
        ps, n_c = inputs.small_set(5), 4
    else:
        ps = inputs.clustered_set(20000, 7, f_blob=0.4, sigma=0.05)
        n_c = int(np.floor(1.0 / (1.825742 * ps.h.max())))
    rec = inputs.pack_aos(ps, "f32")
    for prec in (sph.precision(), sph.precision("f16", "bf16", "f16", 12, 3, 0),
                 sph.precision("f16", "bf16", "f16", 12, 3, 0, anchor=3)):
        dev = Pipeline(rec, n_c, prec=prec)
        dev.bin()
        dev.convert("full")
        host = Pipeline(rec, n_c, prec=prec)
        nbytes = sph.host_staging_size(ps.n, n_c, "full", prec)
        staging = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
        sph.convert_host(rec, host.layout, host.cells, "full", host.soa, staging, nthreads=4)
        torch.cuda.synchronize()
        for name in ("cell_start", "perm", "cell", "hmax"):
            a, b = getattr(dev.cells, name), getattr(host.cells, name)
            assert torch.equal(a.view(torch.uint8), b.view(torch.uint8)), name
        names = ["OFF_X", "OFF_Y", "OFF_Z", "VQ_X", "VQ_Y", "VQ_Z", "M", "H", "U",
                 "X_X", "X_Y", "X_Z", "V_X", "V_Y", "V_Z", "UK"]
        for name in names + (["ANC"] if prec.pos_anchor >= 2 else []):
            a, b = dev.soa[name], host.soa[name]
            assert torch.equal(a.view(torch.uint8), b.view(torch.uint8)), name
        for p in (dev, host):
            p.density()
            p.force()
        torch.cuda.synchronize()
        for name in ("RHO", "F", "NNGB", "A_X", "A_Y", "A_Z", "DU", "VSIG", "NFORCE"):
            a, b = dev.soa[name], host.soa[name]
            assert torch.equal(a.view(torch.uint8), b.view(torch.uint8)), name


def _merge_group(counts, n_c, ti, merge, occ, c):
    """Size of the merged group cell c starts (0 inside another cell's
    group): cells of one 4-cell brick row along x, grouped greedily from the
    row's first cell; a cell joins when it is non-empty, in the occupancy
    class, holds at most ti particles, and the group stays within `merge`
    cells and ti particles."""
    cx, cy, cz = c % n_c, (c // n_c) % n_c, c // (n_c * n_c)
    x0 = cx - cx % 4
    row = [int(counts[x + n_c * (cy + n_c * cz)]) for x in range(x0, min(x0 + 4, n_c))]
    ok = [0 < k <= ti and occ[0] <= k < occ[1] for k in row]
    l = 0
    while l < len(row):
        m = 1
        if ok[l]:
            tot = row[l]
            while l + m < len(row) and m < merge and ok[l + m] and tot + row[l + m] <= ti:
                tot += row[l + m]
                m += 1
        if cx - x0 == l:
            return m
        if cx - x0 < l + m:
            return 0
        l += m
    return 1


def _worklist_reference(start, n, n_c, ti, merge=1, occ=(0, 2 ** 31 - 1)):
    """Items and XCD range boundaries of the work list, rebuilt on the host
    from the cell table: items (cell, first slot) with the cells of the
    occupancy class in brick order; with merge > 1 a cell of at most ti
    particles instead carries one item (cell | (m - 1) << 29, its first
    slot) if it starts a merged group of m cells and none inside one. The
    cost of a cell is ceil(count * min(count of its 27 cells, 27 * 64) /
    4096), clamped so the sum fits in int32; range q starts at the first
    item of the first cell (in brick order) whose cost prefix reaches
    ceil(q * total / 8)."""
    C = n_c ** 3
    order = brick_order(n_c)
    counts = np.diff(start).astype(np.int64)
    cls = np.where((counts >= occ[0]) & (counts < occ[1]), counts, 0)
    items, npos = [], []
    for c in order:
        k = int(cls[c])
        if merge > 1 and 0 < k <= ti:
            m = _merge_group(counts, n_c, ti, merge, occ, int(c))
            if m > 0:
                items.append((int(c) | ((m - 1) << 29), int(start[c])))
            npos.append(1 if m > 0 else 0)
        else:
            items += [(int(c), f) for f in range(start[c], start[c] + k, ti)]
            npos.append((k + ti - 1) // ti)
    grid = counts.reshape(n_c, n_c, n_c)
    nb = sum(np.roll(grid, (dz, dy, dx), axis=(0, 1, 2))
             for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)).reshape(-1)
    cap = (2 ** 31 - 1) // (C + 1)
    cost = np.minimum((cls * np.minimum(nb, 27 * 64) + 4095) >> 12, cap)[order]
    prefix = np.concatenate([[0], np.cumsum(cost)])
    pos = np.concatenate([[0], np.cumsum(npos)])
    total = len(items)
    bounds = [0]
    for q in range(1, 8):
        target = (int(prefix[-1]) * q + 7) // 8
        c = int(np.searchsorted(prefix, target, side="left"))
        bounds.append(min(int(pos[c]), total))
    bounds.append(total)
    return np.array(items, np.int32).reshape(-1, 2), np.array(bounds, np.int32)


def _read_worklist(w, n, n_c):
    buf = w.buf.cpu().numpy()
    meta = buf[64:104].view(np.int32)
    cap = (n + (w.ti - 1) * min(n_c ** 3, n)) // w.ti + 1
    items = buf[len(buf) - 8 * cap:].view(np.int32).reshape(-1, 2)[:meta[0]]
    return items, meta, cap


@pytest.mark.parametrize("ti", [16, 64, 128])
def test_worklist_bit_exact(sph, ti):
    import torch
    from paper_2512_05516_amd.pipeline import Pipeline
    ps = inputs.clustered_set(30000, 5, f_blob=0.5, sigma=0.05)
    n_c = int(np.floor(1.0 / (1.825742 * ps.h.max())))
    rec = inputs.pack_aos(ps, "f32")
    pipe = Pipeline(rec, n_c, til=sph.tile(ti, 256 // ti), sched="grid")
    pipe.bin()
    torch.cuda.synchronize()
    start = pipe.cells.cell_start.cpu().numpy()
    items_ref, bounds_ref = _worklist_reference(start, ps.n, n_c, ti)
    items, meta, cap = _read_worklist(pipe.work, ps.n, n_c)
    assert len(items_ref) <= cap
    assert meta[0] == len(items_ref)
    assert np.array_equal(items, items_ref)
    assert np.array_equal(meta[1:10], bounds_ref)
    assert np.all(np.diff(bounds_ref) >= 0)


@pytest.mark.parametrize("ti,merge,occ", [(64, 4, (0, 2 ** 31 - 1)), (32, 4, (0, 24)),
                                          (64, 2, (0, 2 ** 31 - 1)), (16, 3, (0, 48))])
def test_worklist_merged_bit_exact(sph, ti, merge, occ):
    """Merged work items (max_cells > 1) against the host rebuild, bit for
    bit, and as a partition: every slot of the class's cells lies in exactly
    one item, an item covers at most ti slots, and a merged item's cells are
    consecutive along x within one brick row."""
    import torch
    ps = inputs.clustered_set(30000, 5, f_blob=0.5, sigma=0.05)
    keep = ~((ps.x[:, 0] > 0.30) & (ps.x[:, 0] < 0.52))
    ps = ps.subset(np.nonzero(keep)[0])
    n_c = 13                      # partial bricks at the upper box edge
    cells = sph.DeviceCells(ps.n, n_c, "cuda")
    aos = torch.from_numpy(inputs.pack_aos(ps, "f32").view(np.uint8).reshape(-1).copy()).cuda()
    ws = torch.empty(sph.bin_workspace_size(ps.n, n_c), dtype=torch.uint8, device="cuda")
    sph.bin(aos, sph.layout_from_dtype(inputs.AOS_F32), cells, ws)
    w = sph.DeviceWork(ps.n, n_c, ti, "cuda", "grid", max_cells=merge)
    sph.worklist(cells, w, None, occ)
    torch.cuda.synchronize()
    start = cells.cell_start.cpu().numpy()
    items_ref, bounds_ref = _worklist_reference(start, ps.n, n_c, ti, merge, occ)
    items, meta, cap = _read_worklist(w, ps.n, n_c)
    assert (items_ref[:, 0] >> 29).max() > 0          # some items do merge
    assert meta[0] == len(items_ref)
    assert np.array_equal(items, items_ref)
    assert np.array_equal(meta[1:10], bounds_ref)
    counts = np.diff(start)
    covered = np.zeros(ps.n, np.int32)
    for v, f in items:
        c, m = int(v) & ((1 << 29) - 1), (int(v) >> 29) + 1
        if m > 1:
            assert c % n_c + m - 1 < n_c and (c % n_c) // 4 == (c % n_c + m - 1) // 4
            assert f == start[c] and start[c + m] - f <= ti
            covered[f:start[c + m]] += 1
        else:
            covered[f:min(f + ti, start[c + 1])] += 1
    in_cls = np.repeat((counts >= occ[0]) & (counts < occ[1]), counts)
    assert np.array_equal(covered, in_cls.astype(np.int32))


# ---------------------------------------------------------------------------
# density / force against the FP64 oracle
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind,mode", [("f32", {}), ("f64", {}),
                                       ("f32", {"sub_bits": 1, "sched": "dynamic"}),
                                       ("f64", {"sub_bits": 2, "sched": "static"}),
                                       ("f32", {"sched": "grid"}),
                                       ("f32", {"sub_bits": 1})])
def test_small_lattice_parity(sph, orc, kind, mode):
    ps = inputs.small_set(1)                        # 4,096 particles, shuffled order
    n_c = 4
    pipe = run_gpu(ps, n_c, kind, **mode)
    assert pipe.status() == 0
    got = gpu_fields(pipe)
    ref = inputs.unpack_aos(inputs.pack_aos(ps, kind))
    got["h"] = ref.h
    d, f = oracle_step(orc, ps, n_c)                # FP64, unrounded inputs
    assert_counts(orc, got["nngb"], got["nforce"], d["nngb"], f["nforce"], ps, n_c,
                  min_clear=0.98, tag=f"S/{kind}/{mode}")
    check_fp32(got, d, f, tag=f"S/{kind}/{mode}")


@pytest.fixture(scope="module")
def dense_blobs(orc):
    # compact blobs (sigma 0.01, 80 % of 40,000 particles) in cells sized by the
    # background h: a dozen cells above 1,024 particles, split at sub-cell
    # depth 3 (more than 2 x 8^3), whose chunks reach hundreds of sub-cell
    # ranges (several range-table batches per chunk) and, for the force, whose
    # neighbour cells hold background h, thousands of candidates (many LDS
    # batches, so the ranges are placed by class)
    ps = inputs.clustered_set(40000, 11, f_blob=0.8, sigma=0.01)
    n_c = int(np.floor(1.0 / (orc.GAMMA_K * ps.h.max())))
    ref = inputs.unpack_aos(inputs.pack_aos(ps, "f32"))
    d, f = oracle_step(orc, ref, n_c)
    return ps, ref, n_c, d, f


@pytest.fixture(scope="module")
def ragged(orc):
    # clustered set with a slab cut out: empty cells, nearly empty cells, cells
    # spanning several chunks (ragged tails), uneven h
    ps = inputs.clustered_set(30000, 5, f_blob=0.5, sigma=0.05)
    keep = ~((ps.x[:, 0] > 0.30) & (ps.x[:, 0] < 0.52))
    ps = ps.subset(np.nonzero(keep)[0])
    n_c = int(np.floor(1.0 / (orc.GAMMA_K * ps.h.max())))
    ref = inputs.unpack_aos(inputs.pack_aos(ps, "f32"))
    d, f = oracle_step(orc, ref, n_c)
    return ps, ref, n_c, d, f


@pytest.mark.parametrize("ti,k,bits,sched", [(16, 4, 3, "static"), (64, 1, 3, "grid"),
                                             (32, 2, 3, None), (128, 2, 3, "dynamic"),
                                             (64, 2, 2, "grid")])
def test_dense_blob_sub_cells_parity(sph, orc, dense_blobs, ti, k, bits, sched):
    ps, ref, n_c, d, f = dense_blobs
    pipe = run_gpu(ps, n_c, "f32", til=sph.tile(ti, k), sub_bits=bits, sched=sched)
    assert pipe.status() == 0
    counts = np.diff(pipe.cells.cell_start.cpu().numpy())
    assert (counts > 2 * 8 ** bits).sum() >= 5         # cells split into sub-cell ranges
    got = gpu_fields(pipe)
    got["h"] = ref.h
    assert_counts(orc, got["nngb"], got["nforce"], d["nngb"], f["nforce"], ref, n_c,
                  tag=f"dense/{ti}x{k}")
    check_fp32(got, d, f, tag=f"dense/{ti}x{k}/sub{bits}/{sched or 'cells'}")


@pytest.mark.parametrize("ti,k,bits,sched", [(64, 4, 0, None), (32, 8, 0, None),
                                             (128, 2, 0, None), (64, 2, 0, None),
                                             (64, 1, 0, None), (64, 4, 2, "dynamic"),
                                             (32, 8, 3, "static"), (16, 16, 2, "grid"),
                                             (128, 2, 1, "dynamic"), (64, 1, 3, "grid"),
                                             (64, 4, 1, "static"), (32, 8, 2, "grid"),
                                             (16, 4, 0, None), (32, 2, 2, "grid"),
                                             (16, 4, 3, "static")])
def test_ragged_clustered_parity(sph, orc, ragged, ti, k, bits, sched):
    ps, ref, n_c, d, f = ragged
    pipe = run_gpu(ps, n_c, "f32", til=sph.tile(ti, k), sub_bits=bits, sched=sched)
    assert pipe.status() == 0
    counts = np.diff(pipe.cells.cell_start.cpu().numpy())
    assert counts.min() == 0 and counts.max() > 2 * ti
    got = gpu_fields(pipe)
    got["h"] = ref.h
    assert_counts(orc, got["nngb"], got["nforce"], d["nngb"], f["nforce"], ref, n_c,
                  tag=f"clustered/{ti}x{k}")
    check_fp32(got, d, f, tag=f"clustered/{ti}x{k}/sub{bits}/{sched or 'cells'}")


def test_autotuned_config_parity(sph, orc, ragged, tmp_path):
    from paper_2512_05516_amd import tune
    ps, ref, n_c, d, f = ragged
    rec = inputs.pack_aos(ps, "f32")
    cache = str(tmp_path / "tune.json")
    choice = tune.tune(rec, n_c, sub_bits=(0, 2), reps=1, cache_path=cache)
    assert not choice["cached"]
    assert len(choice["table"]) == 2 * 2 * len(sph.tune_candidates())
    assert all(r["ms"] > 0 for r in choice["table"])
    again = tune.tune(rec, n_c, sub_bits=(0, 2), reps=1, cache_path=cache)
    assert again["cached"] and again["density"] == choice["density"]
    pipe = run_gpu(ps, n_c, "f32", **tune.pipeline_kwargs(choice))
    assert pipe.status() == 0
    got = gpu_fields(pipe)
    got["h"] = ref.h
    assert_counts(orc, got["nngb"], got["nforce"], d["nngb"], f["nforce"], ref, n_c, tag="tuned")
    check_fp32(got, d, f, tag=f"clustered/tuned/{tune.describe(choice)}")


def test_perfect_lattice_closed_form_gpu(sph, orc):
    ps = inputs.lattice_set(16, 0, perfect=True, order="shuffled")
    pipe = run_gpu(ps, 4)
    got = gpu_fields(pipe)
    assert np.all(got["nngb"] == 57) and np.all(got["nforce"] == 56)
    rho_cf = 1.0039808                     # a^-3 sum_k w(|k|/a), pinned on the oracle side
    assert np.max(np.abs(got["rho"] - rho_cf)) < 2e-6
    assert np.max(np.abs(got["wcount"] - 48.186135)) < 1e-3
    # forces vanish by symmetry; the FP32 residue is bounded relative to the
    # size of one pair's pressure term m 2 P/rho^2 / H^4
    H = 1.825742 * ps.h[0]
    pair = ps.m[0] * 2 * got["P"][0] / got["rho"][0] ** 2 / H ** 4
    assert np.max(np.abs(got["a"])) < 1e-5 * pair


# reduced storage: (pos, vel, mhu, scales, position anchor); the first is the
# benchmark's mixed format with positions anchored at sub-cell centres
SUB2 = 3      # SPH_ANCHOR_SUB(2)
RPRECS = [("f16", "bf16", "f16", (12, 3, 0), SUB2), ("f16", "f16", "f16", (21, 6, -1), SUB2),
          ("bf16", "bf16", "bf16", (0, 0, 0), SUB2), ("f16", "bf16", "f16", (12, 3, 0), 0),
          ("bf16", "f16", "bf16", (0, 0, 0), 1), ("f16", "f16", "f16", (12, 3, 0), 2)]


@pytest.mark.parametrize("pos,vel,mhu,scales,anchor", RPRECS)
def test_reduced_precision(sph, orc, pos, vel, mhu, scales, anchor):
    """Kernel arithmetic on the stored values against the oracle on the same
    dequantised inputs (counts against FP64 brute force, sums at the FP32
    bar); the storage error against FP64 on the unrounded inputs gated at
    the stated tolerances: FP16 positions, h, m anchored at sub-cell
    centres keep rho and a within 2e-3, BF16 velocities du/dt within 8e-3."""
    ps = inputs.small_set(2)
    n_c = 4
    prec = sph.precision(pos, vel, mhu, *scales, anchor=anchor)
    pipe = run_gpu(ps, n_c, "f32", prec=prec)
    assert pipe.status() == 0
    got = gpu_fields(pipe)
    ref = inputs.unpack_aos(inputs.pack_aos(ps, "f32"))
    q = orc.dequantise_set(ref, n_c, pos, vel, mhu, scales, anchor=anchor)
    got["h"] = q.h
    dq, fq = oracle_step(orc, q, n_c)
    assert_counts(orc, got["nngb"], got["nforce"], dq["nngb"], fq["nforce"], q, n_c,
                  min_clear=0.98, tag=f"{pos}/{vel}/{mhu}/{anchor}")
    check_fp32(got, dq, fq, tol=2e-5, tag=f"{pos}/{vel}/{mhu}/{anchor} vs dequantised")
    d, f = oracle_step(orc, ps, n_c)
    e = {"rho": max_rel(got["rho"], d["rho"]), "a": rel_rmse(got["a"], f["a"]),
         "du": rel_rmse(got["du"], f["du"])}
    print(f"storage error vs FP64 {pos}/{vel}/{mhu}/anchor {anchor}:",
          {k: f"{v:.2e}" for k, v in e.items()})
    if anchor == SUB2 and pos == "f16" and mhu == "f16":
        assert e["rho"] <= 2e-3 and e["a"] <= 2e-3, e
        assert e["du"] <= (8e-3 if vel == "bf16" else 2e-3), e
    if anchor == SUB2 and pos == "bf16":
        assert e["rho"] <= 8e-3 and e["du"] <= 8e-3, e


def test_coincident_positions(sph, orc):
    """Particles at the same stored position (exact duplicates, and pairs
    closer than an FP16 step, which collide once positions are stored in
    FP16): the pair counts, exerts no force and its signal velocity is
    c_i + c_j, as the oracle defines it; FP32 and FP16 storage against the
    oracle on the same stored values."""
    base = inputs.small_set(5)
    rng = np.random.default_rng(8)
    src = rng.choice(base.n, 40, replace=False)
    dup = base.subset(src)
    dup.x[:20] = base.x[src[:20]]                            # exact duplicates
    dup.x[20:] = base.x[src[20:]] + rng.uniform(-1, 1, (20, 3)) * 2e-9   # below an FP16 step
    dup.v = rng.normal(0.0, 0.05, (40, 3))
    ps = inputs.ParticleSet(np.concatenate([base.x, dup.x]), np.concatenate([base.v, dup.v]),
                            np.concatenate([base.m, dup.m]), np.concatenate([base.h, dup.h]),
                            np.concatenate([base.u, dup.u]))
    n_c = 4
    ref = inputs.unpack_aos(inputs.pack_aos(ps, "f32"))
    for pos, anchor in (("f32", 0), ("f16", SUB2)):
        prec = sph.precision(pos, "f32", "f32", anchor=anchor)
        pipe = run_gpu(ps, n_c, "f32", prec=prec)
        assert pipe.status() == 0
        got = gpu_fields(pipe)
        q = orc.dequantise_set(ref, n_c, pos, "f32", "f32", anchor=anchor)
        xq = q.x
        same = np.array([np.all(xq[i] == xq[j]) for i, j in zip(src, base.n + np.arange(40))])
        assert same[:20].all() and (pos == "f32" or same.sum() >= 30), (pos, same.sum())
        dq, fq = oracle_step(orc, q, n_c)
        assert np.all(np.isfinite(fq["a"])) and np.all(np.isfinite(got["a"]))
        got["h"] = q.h
        assert_counts(orc, got["nngb"], got["nforce"], dq["nngb"], fq["nforce"], q, n_c,
                      min_clear=0.97, tag=f"coincident/{pos}")
        check_fp32(got, dq, fq, tol=2e-5, tag=f"coincident/{pos}")


# ---------------------------------------------------------------------------
# AoS == SoA, determinism, kick/drift, reductions, edge cases
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mode", [{}, {"sub_bits": 2, "sched": "dynamic"},
                                  {"sub_bits": 1, "sched": ("grid", "static")},
                                  {"sub_bits": 1, "sched": "grid",
                                   "split": {"density": (32, (32, 2), "grid", 4),
                                             "force": (32, (64, 1), "grid", 4)}}])
def test_aos_equals_soa_bitwise(sph, mode):
    from paper_2512_05516_amd.pipeline import Pipeline
    ps = inputs.clustered_set(20000, 9, f_blob=0.4, sigma=0.05)
    rec = inputs.pack_aos(ps, "f32")
    n_c = int(np.floor(1.0 / (1.825742 * ps.h.max())))
    a = Pipeline(rec, n_c, **mode)
    b = Pipeline(rec, n_c, **mode)
    for _ in range(2):
        a.soa_step(1e-3, 1e-3)
        b.aos_step(1e-3, 1e-3)
    ra, rb = a.records(), b.records()
    for k in ("x", "v", "u", "a", "du", "rho", "wcount", "rho_dh", "f", "P", "c", "vsig",
              "nngb", "nforce"):
        assert np.ascontiguousarray(ra[k]).tobytes() == np.ascontiguousarray(rb[k]).tobytes(), k
    # the FP64 reductions of the last step: over the records (sph_reduce_aos)
    # the same sums as over the FP32 SoA (sph_reduce), bit for bit
    assert a.red_out.cpu().numpy().tobytes() == b.red_out.cpu().numpy().tobytes()
    assert b.red_out.cpu().numpy()[6] == rb["nngb"].sum()


@pytest.mark.parametrize("kind", ["f32", "f64"])
def test_aos_steps_records_kinds_and_kept_cells(sph, kind):
    """Plain-AoS steps on FP32 and FP64 records (the latter the small
    configuration's record): the records and the FP64 sums equal those of
    the SoA path bit for bit, and keeping the cell list between AoS steps
    (the records' kick/drift counting particles that leave their cell or
    sub-cell) gives the records of rebinning every step; the list is kept
    over kick-only steps and rebuilt after a drift."""
    from paper_2512_05516_amd.pipeline import Pipeline
    ps = inputs.clustered_set(20000, 6, f_blob=0.4, sigma=0.05)
    rec = inputs.pack_aos(ps, kind)
    n_c = int(np.floor(1.0 / (1.825742 * ps.h.max())))
    kw = dict(sub_bits=1, sched="grid")
    soa, aos = Pipeline(rec, n_c, **kw), Pipeline(rec, n_c, **kw)
    keep = Pipeline(rec, n_c, keep_cells=True, **kw)
    rebuilt = []
    for dt_drift in (0.0, 0.0, 2e-3, 0.0):
        soa.soa_step(1e-4, dt_drift)
        aos.aos_step(1e-4, dt_drift)
        keep.aos_step(1e-4, dt_drift)
        rebuilt.append(int(keep.cells.rebin[1].item()))
        ra, rb, rk = soa.records(), aos.records(), keep.records()
        for k in ("x", "v", "u", "a", "du", "rho", "wcount", "rho_dh", "f", "P", "c", "vsig",
                  "nngb", "nforce"):
            assert np.ascontiguousarray(ra[k]).tobytes() == np.ascontiguousarray(rb[k]).tobytes(), k
        assert rb.tobytes() == rk.tobytes(), (dt_drift, rebuilt)
        assert soa.red_out.cpu().numpy().tobytes() == aos.red_out.cpu().numpy().tobytes()
    # built by the first step, kept after kick-only steps, rebuilt after the drift
    assert rebuilt == [1, 0, 0, 1], rebuilt
    assert aos.status() == 0 and keep.status() == 0


@pytest.mark.parametrize("mode", [{}, {"sub_bits": 1, "sched": "dynamic"}])
def test_deterministic(sph, mode):
    ps = inputs.clustered_set(30000, 4, f_blob=0.5, sigma=0.05)
    n_c = int(np.floor(1.0 / (1.825742 * ps.h.max())))
    r1 = run_gpu(ps, n_c, **mode).records()
    r2 = run_gpu(ps, n_c, **mode).records()
    assert r1.tobytes() == r2.tobytes()


def test_kick_drift_parity(sph, orc):
    ps = inputs.small_set(6)
    n_c = 4
    dt = 2e-3
    pipe = run_gpu(ps, n_c, kick=(dt, dt))
    got = gpu_fields(pipe)
    ref = inputs.unpack_aos(inputs.pack_aos(ps, "f32"))
    d, f = oracle_step(orc, ref, n_c)
    x1, v1, u1 = orc.kick_drift(ref.x, ref.v, ref.u, f["a"], f["du"], dt, dt)
    dv = np.abs(got["v"] - v1).max()
    assert dv <= 1e-5 * np.abs(f["a"]).max() * dt + 1e-8
    dx = np.abs(got["x"] - x1)
    dx = np.minimum(dx, 1 - dx).max()
    assert dx <= 1e-7 * dt
    assert np.abs(got["u"] - u1).max() <= 1e-6


def test_kick_drift_wraps_and_counts_moves(sph, orc):
    import torch
    ps = inputs.small_set(7)
    n_c = 4
    ps.v = ps.v * 0 + np.array([0.3, -0.2, 0.05])     # large uniform drift
    dt = 0.3
    pipe = run_gpu(ps, n_c)
    pipe.moved.zero_()
    pipe.kick_drift(0.0, dt)
    pipe.writeback("kick")
    got = pipe.records()
    x1 = ps.x + ps.v.astype(np.float32).astype(np.float64) * dt
    x1 -= np.floor(x1)
    assert np.all((got["x"] >= 0) & (got["x"] < 1))
    assert np.max(np.abs(got["x"] - x1)) < 1e-15
    c0 = orc.bin_cells(ps.x, n_c)[0]
    c1 = orc.bin_cells(x1, n_c)[0]
    torch.cuda.synchronize()
    assert pipe.moved.item() == int((c0 != c1).sum())


def test_reduce_fp64(sph):
    import math
    ps = inputs.small_set(8)
    pipe = run_gpu(ps, 4)
    out = pipe.red_out.cpu().numpy()
    got = gpu_fields(pipe)
    m = ps.m.astype(np.float32).astype(np.float64)
    # exactly rounded FP64 sums of the same FP32 values (math.fsum)
    va = (got["v"] * got["a"]).sum(1)
    ref = [math.fsum(m * got["a"][:, 0]), math.fsum(m * got["a"][:, 1]),
           math.fsum(m * got["a"][:, 2]), math.fsum(m * (va + got["du"])),
           math.fsum(m * np.linalg.norm(got["a"], axis=1)),
           math.fsum(m * (np.abs(va) + np.abs(got["du"])))]
    assert np.allclose(out[:6], ref, rtol=1e-12, atol=1e-12 * ref[4])
    assert out[6] == got["nngb"].sum() and out[7] == got["nforce"].sum()
    # FP32 pair terms are evaluated twice, so momentum is conserved to ~FP32
    assert np.linalg.norm(out[:3]) / out[4] < 1e-5
    assert abs(out[3]) / out[5] < 1e-5


def test_edge_cases(sph, orc):
    import torch
    # empty set: every stage is a no-op
    empty = inputs.ParticleSet(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), np.zeros(0),
                               np.zeros(0))
    pipe = run_gpu(empty, 3, kick=(1e-4, 1e-4))
    assert pipe.cells.cell_start.cpu().numpy().sum() == 0
    # one particle: only the self pair
    one = inputs.ParticleSet(np.array([[0.3, 0.6, 0.9]]), np.zeros((1, 3)), np.array([0.5]),
                             np.array([0.1]), np.array([1.0]))
    got = gpu_fields(run_gpu(one, 3))
    assert got["nngb"][0] == 1 and got["nforce"][0] == 0
    H = 1.825742 * 0.1
    assert abs(got["rho"][0] / (0.5 * (8 / np.pi) / H ** 3) - 1) < 1e-6
    assert np.all(got["a"] == 0)
    # smoothing length beyond the cell side raises the status flag
    ps = inputs.small_set(1)
    ps.h = ps.h * 2.0
    pipe = run_gpu(ps, 4)
    assert pipe.status() & sph.FLAG_H_TOO_LARGE


# ---------------------------------------------------------------------------
# full size, in the launch configuration the benchmark times
# ---------------------------------------------------------------------------

def test_full_size_medium(sph, orc):
    """2,097,152 particles (128^3 lattice, FP32 records) in the tiling the
    benchmark's autotuner chooses: binning bit-exact, every neighbour count
    exact, values on a seeded sample of 4,096 particles within the FP32 bar."""
    from paper_2512_05516_amd import tune
    ps = inputs.medium_set(2)
    n_c = 32
    rec = inputs.pack_aos(ps, "f32")
    choice = tune.tune(rec, n_c, reps=3, cache_path=None)
    kw = tune.pipeline_kwargs(choice)
    pipe = run_gpu(ps, n_c, "f32", **kw)
    assert pipe.status() == 0
    ref = inputs.unpack_aos(rec)
    _, ostart, operm, _ = orc.bin_cells(ref.x, n_c)
    assert np.array_equal(pipe.cells.cell_start.cpu().numpy(), ostart)
    if kw["sub_bits"]:
        _, _, operm = orc.bin_sub(ref.x, n_c, kw["sub_bits"])
    assert np.array_equal(pipe.cells.perm.cpu().numpy(), operm)
    got = gpu_fields(pipe)
    # every count against the FP64 counts (the force loop's over all particles)
    d = orc.density(ps, n_c=n_c)
    f_all = orc.force(ps, d, n_c=n_c)
    assert_counts(orc, got["nngb"], got["nforce"], d["nngb"], f_all["nforce"], ps, n_c,
                  min_clear=0.98, tag="M")
    nd, nf = got["nngb"], got["nforce"]
    sel = np.sort(np.random.default_rng(11).choice(ps.n, 4096, replace=False)).astype(np.int32)
    f = {k: v[sel] for k, v in f_all.items()}
    sub = {k: v[sel] for k, v in got.items()}
    sub["h"] = ref.h[sel]
    dsub = {k: v[sel] for k, v in d.items()}
    check_fp32(sub, dsub, f, tag=f"M/sample/{tune.describe(choice)}")
    # FP64 reductions over all slots equal the sums of the counts
    out = pipe.red_out.cpu().numpy()
    assert out[6] == nd.sum() and out[7] == nf.sum()


@pytest.fixture(scope="module")
def m_tiling(sph):
    """The benchmark's tiling of the 128^3 set (autotuned on FP32 storage,
    used for every storage format of that set)."""
    from paper_2512_05516_amd import tune
    rec = inputs.pack_aos(inputs.medium_set(2), "f32")
    return tune.pipeline_kwargs(tune.tune(rec, 32, reps=2, cache_path=None))


@pytest.mark.parametrize("fmt", [("f16", "bf16", "f16", (21, 7, 0)), ("f16", "f16", "f16", (21, 7, 0)),
                                 ("bf16", "bf16", "bf16", (0, 0, 0))],
                         ids=["fp16_store", "fp16_all", "bf16_all"])
def test_full_size_reduced(sph, orc, m_tiling, fmt):
    """The 128^3 set with reduced-precision storage as the benchmark runs it
    (positions as offsets from sub-cell centres; the mixed FP16/BF16 format,
    all-FP16 and all-BF16), in the benchmark's tiling: on a seeded sample of
    8,192 particles, counts against FP64 brute force and values against the
    oracle on the dequantised inputs at the kernels' bar, and the storage
    error against FP64 on the unrounded inputs within the stated tolerances
    (FP16 positions: rho and a 2e-3; du/dt 2e-3, or 8e-3 with BF16
    velocities; all-BF16 8e-3)."""
    pos, vel, mhu, scales = fmt
    ps = inputs.medium_set(2)
    n_c = 32
    prec = sph.precision(pos, vel, mhu, *scales, anchor=SUB2)
    pipe = run_gpu(ps, n_c, "f32", prec=prec, **m_tiling)
    assert pipe.status() == 0
    got = gpu_fields(pipe)
    ref = inputs.unpack_aos(inputs.pack_aos(ps, "f32"))
    q = orc.dequantise_set(ref, n_c, pos, vel, mhu, scales, anchor=SUB2)
    sel = np.sort(np.random.default_rng(21).choice(ps.n, 8192, replace=False)).astype(np.int32)
    d, f = _oracle_at(orc, q, n_c, sel)
    tag = "/".join((pos, vel, mhu))
    assert_counts(orc, got["nngb"][sel], got["nforce"][sel], d["nngb"], f["nforce"], q, n_c,
                  sel=sel, min_clear=0.98, tag=f"R/{tag}")
    sub = {k: v[sel] for k, v in got.items()}
    sub["h"] = q.h[sel]
    check_fp32(sub, d, f, tol=2e-5, tag=f"R/{tag} vs dequantised")
    d0, f0 = _oracle_at(orc, ref, n_c, sel)
    e = {"rho": max_rel(sub["rho"], d0["rho"]), "a": rel_rmse(sub["a"], f0["a"]),
         "du": rel_rmse(sub["du"], f0["du"])}
    print(f"R/{tag} storage error vs FP64:", {k: f"{v:.2e}" for k, v in e.items()})
    if pos == "f16":
        assert e["rho"] <= 2e-3 and e["a"] <= 2e-3, e
        assert e["du"] <= (8e-3 if vel == "bf16" else 2e-3), e
    else:
        assert e["rho"] <= 8e-3 and e["a"] <= 8e-3 and e["du"] <= 8e-3, e


@pytest.fixture(scope="module")
def k_state(sph):
    """The clustered 4,194,304-particle set as the benchmark times it: h from
    the density iteration on the GPU (settle_h, tol 1e-4), then cells as
    small as the largest support radius allows."""
    from paper_2512_05516_amd.pipeline import settle_h
    ps = inputs.clustered_k_set(3)
    rec, n_c, info = settle_h(inputs.pack_aos(ps, "f32"), tol=1e-4, max_iter=30, room=1.6)
    assert info["not_converged"] == 0
    return rec, n_c


def _oracle_at(orc, ps, n_c, sel):
    """Oracle density and force at the particles `sel` of ps (density also
    at their force neighbours, which the force reads)."""
    need = _force_neighbours(ps, n_c, sel, orc.GAMMA_K)
    dn = orc.density(ps, n_c=n_c, sel=need)
    d = {k: np.full(ps.n, np.nan) for k in ("rho", "wcount", "rho_dh", "f", "P", "c")}
    d["nngb"] = np.full(ps.n, -1, np.int32)
    for k in d:
        d[k][need] = dn[k]
    f = orc.force(ps, d, n_c=n_c, sel=sel)
    return {k: v[sel] for k, v in d.items()}, f


@pytest.mark.parametrize("storage", ["fp32", "fp16_store"])
def test_full_size_clustered(sph, orc, k_state, storage):
    """The benchmark's clustered configuration: 4,194,304 particles with h
    from the GPU iteration, occupancy up to about 2,000 per cell, in the
    tiling (and occupancy split) the autotuner picks for each storage:
    binning bit-exact; on a seeded sample of background particles and of
    particles in the most crowded cells, counts against FP64 brute force
    and values against the oracle on the stored values at the kernels' bar;
    for FP16 storage also the storage error against FP64 on the unrounded
    inputs within the stated 2e-3 (rho, a) and 8e-3 (du/dt, BF16 v)."""
    from paper_2512_05516_amd import tune
    rec, n_c = k_state
    ref = inputs.unpack_aos(rec)
    if storage == "fp32":
        prec, fm, tol = sph.precision(), None, FP32_TOL
    else:
        fm = ("f16", "bf16", "f16", (22, 7, 0))
        prec, tol = sph.precision(*fm[:3], *fm[3], anchor=SUB2), 2e-5
    choice = tune.tune(rec, n_c, prec=prec, sub_bits=(2,), reps=2, cache_path=None)
    pipe = run_gpu(ref, n_c, "f32", prec=prec, **tune.pipeline_kwargs(choice))
    assert pipe.status() == 0
    _, ostart, _, _ = orc.bin_cells(ref.x, n_c)
    assert np.array_equal(pipe.cells.cell_start.cpu().numpy(), ostart)
    occ = np.diff(ostart)
    assert 1500 < occ.max() < 2600 and occ.min() <= 16, (occ.min(), occ.max())
    got = gpu_fields(pipe)
    rng = np.random.default_rng(12)
    cell_of = np.minimum((ref.x * n_c).astype(int), n_c - 1) @ np.array([1, n_c, n_c * n_c])
    crowded = np.nonzero(occ[cell_of] > 0.6 * occ.max())[0]
    sel = np.unique(np.concatenate([rng.choice(ref.n, 512, replace=False),
                                    rng.choice(crowded, 256, replace=False)])).astype(np.int32)
    q = orc.dequantise_set(ref, n_c, *fm[:3], fm[3], anchor=SUB2) if fm else ref
    d, f = _oracle_at(orc, q, n_c, sel)
    assert np.all(np.isfinite(f["a"])) and np.all(np.isfinite(f["du"]))
    assert_counts(orc, got["nngb"][sel], got["nforce"][sel], d["nngb"], f["nforce"], q, n_c,
                  sel=sel, tag=f"K/{storage}")
    sub = {k: v[sel] for k, v in got.items()}
    sub["h"] = q.h[sel]
    tag = f"K/{storage}/sample/{tune.describe(choice)}"
    check_fp32(sub, d, f, tol=tol, tag=tag)
    if fm:
        d0, f0 = _oracle_at(orc, ref, n_c, sel)
        e = {"rho": max_rel(sub["rho"], d0["rho"]), "a": rel_rmse(sub["a"], f0["a"]),
             "du": rel_rmse(sub["du"], f0["du"])}
        print(tag, "storage error vs FP64:", {k: f"{v:.2e}" for k, v in e.items()})
        assert e["rho"] <= 2e-3 and e["a"] <= 2e-3 and e["du"] <= 8e-3, e


def _force_neighbours(ps, n_c, sel, gamma_k):
    """Indices of sel and of every j with r_ij < max(H_i, H_j) for some i in
    sel (periodic minimum image; candidates from the 27 cells around i)."""
    x, H = np.asarray(ps.x), gamma_k * np.asarray(ps.h)
    cell = np.minimum((x * n_c).astype(int), n_c - 1)
    cid = cell @ np.array([1, n_c, n_c * n_c])
    order = np.argsort(cid, kind="stable")
    start = np.searchsorted(cid[order], np.arange(n_c ** 3 + 1))
    out = [np.asarray(sel)]
    offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    for i in sel:
        c = cell[i]
        cand = np.concatenate([order[start[k]:start[k + 1]] for k in
                               {((c[0] + dx) % n_c) + n_c * (((c[1] + dy) % n_c) +
                                                           n_c * ((c[2] + dz) % n_c))
                                for dx, dy, dz in offs}])
        d = x[cand] - x[i]
        d -= np.rint(d)
        r = np.sqrt((d * d).sum(1))
        out.append(cand[r < np.maximum(H[i], H[cand])])
    return np.unique(np.concatenate(out)).astype(np.int32)


# ---------------------------------------------------------------------------
# truncate_mantissa storage (packed T-bit codes)
# ---------------------------------------------------------------------------

TRUNC_PRECS = [("t20", "t20", "t20", (12, 3, 0)), ("t12", "t14", "t10", (10, 4, 0)),
               ("t27", "t17", "t31", (0, 0, 0)), ("t16", "t32", "t9", (12, 3, 0))]


@pytest.mark.parametrize("kind", ["f32", "f64"])
@pytest.mark.parametrize("pos,vel,mhu,scales", TRUNC_PRECS)
def test_convert_truncated_bit_exact(sph, orc, kind, pos, vel, mhu, scales):
    """Packed codes decode to exactly the oracle's truncated values."""
    import torch
    from paper_2512_05516_amd.pipeline import Pipeline
    ps = inputs.clustered_set(3001, 8, f_blob=0.4, sigma=0.06)   # ragged last tile
    n_c = int(np.floor(1.0 / (orc.GAMMA_K * ps.h.max())))
    rec = inputs.pack_aos(ps, kind)
    ref = inputs.unpack_aos(rec)
    prec = sph.precision(pos, vel, mhu, *scales)
    pipe = Pipeline(rec, n_c, prec=prec)
    pipe.bin()
    pipe.convert("full")
    torch.cuda.synchronize()
    perm = pipe.cells.perm.cpu().numpy()
    _, _, _, off = orc.bin_cells(ref.x, n_c)
    T = lambda s: int(s[1:])
    want = {}
    for a, ax in enumerate("XYZ"):
        want["OFF_" + ax] = (pos, [orc.roundtrip(v, pos) for v in off[perm, a]], 0)
        want["VQ_" + ax] = (vel, [orc.roundtrip(v, vel) for v in ref.v[perm, a]], 0)
    for name, arr, sc in (("M", ref.m, scales[0]), ("H", ref.h, scales[1]), ("U", ref.u, scales[2])):
        want[name] = (mhu, [orc.roundtrip(v, mhu, sc) for v in arr[perm]], sc)
    for name, (fmt, vals, sc) in want.items():
        words = pipe.soa[name].cpu().numpy()
        got = unpack_trunc(words, T(fmt), ps.n).astype(np.float64) * 2.0 ** -sc
        assert np.array_equal(got, np.asarray(vals)), (name, fmt)


@pytest.mark.parametrize("pos,vel,mhu,scales", TRUNC_PRECS)
def test_truncated_storage_parity(sph, orc, pos, vel, mhu, scales):
    """Pair loops on truncated storage: counts against FP64 brute force and
    sums against the oracle, both on the same stored values."""
    ps = inputs.small_set(3)
    n_c = 4
    pipe = run_gpu(ps, n_c, "f32", prec=sph.precision(pos, vel, mhu, *scales))
    assert pipe.status() == 0
    got = gpu_fields(pipe)
    ref = inputs.unpack_aos(inputs.pack_aos(ps, "f32"))
    q = orc.dequantise_set(ref, n_c, pos, vel, mhu, scales)
    got["h"] = q.h
    dq, fq = oracle_step(orc, q, n_c)
    assert_counts(orc, got["nngb"], got["nforce"], dq["nngb"], fq["nforce"], q, n_c,
                  min_clear=0.98, tag=f"trunc {pos}/{vel}/{mhu}")
    check_fp32(got, dq, fq, tol=2e-5, tag=f"{pos}/{vel}/{mhu} vs dequantised")


def test_truncation_error_curve_gpu(sph, orc):
    """Acceleration error of the FP32 kernels on T-bit storage (every field)
    against FP64 on the unrounded inputs, at the size of the paper's
    experiment (a jittered 40^3 lattice, 64,000 particles, one force
    evaluation): at 32 bits the FP32 floor; growing as bits are cut within
    the single and half layouts, about doubling per bit; lower at exactly
    16 bits than at 17 (the switch to the half layout)."""
    ps = inputs.lattice_set(40, 1, order="shuffled")
    n_c = int(np.floor(1.0 / (orc.GAMMA_K * ps.h.max())))
    d0, f0 = oracle_step(orc, ps, n_c)
    e = {}
    for T in (32, 30, 28, 26, 24, 22, 20, 18, 17, 16, 14, 12, 10):
        t = f"t{T}"
        pipe = run_gpu(ps, n_c, "f32", prec=sph.precision(t, t, t, 16, 5, 0))
        assert pipe.status() == 0
        e[T] = rel_rmse(gpu_fields(pipe)["a"], f0["a"])
    print("RMSE(a) vs bits, 64,000 particles:", {T: f"{v:.2e}" for T, v in e.items()})
    assert e[32] < 1e-5
    for a, b in ((30, 32), (28, 30), (26, 28), (24, 26), (22, 24), (20, 22), (18, 20), (17, 18),
                 (14, 16), (12, 14), (10, 12)):
        assert e[a] > e[b], (a, b)
    for a, b in ((24, 26), (22, 24), (20, 22), (18, 20), (12, 14)):
        assert 2.5 < e[a] / e[b] < 6.0, (a, b, e[a] / e[b])      # about 4x per two bits cut
    assert e[16] < e[17]


# ---------------------------------------------------------------------------
# smoothing lengths: h = eta (m / rho(h))^(1/3)
# ---------------------------------------------------------------------------

def _h_max(sph, n_c):
    """The largest FP32 h with (gamma_k h)^2 <= (1/n_c)^2 in FP32 and
    gamma_k h <= 1/n_c exactly."""
    g64 = sph.params().gamma_k
    gk = np.float32(g64)
    s = np.float32(1.0 / n_c)
    h = np.float32(s / gk)
    while (gk * h) * (gk * h) > s * s or g64 * float(h) > 1.0 / n_c:
        h = np.nextafter(h, np.float32(0))
    return float(h)


@pytest.mark.parametrize("which,sched,sub_bits", [("lattice", None, 0), ("clustered", None, 0),
                                                  ("clustered", "grid", 0),
                                                  ("clustered", "grid", 2)])
def test_smoothing_length_matches_oracle(sph, orc, which, sched, sub_bits):
    import torch
    from paper_2512_05516_amd.pipeline import Pipeline
    if which == "lattice":
        ps, n_c = inputs.small_set(2), 4
    else:
        ps = inputs.clustered_set(20000, 6, f_blob=0.4, sigma=0.05)
        n_c = int(np.floor(1.0 / (1.3 * orc.GAMMA_K * ps.h.max())))
    ps.h = ps.h * np.random.default_rng(3).uniform(0.75, 1.3, ps.n)
    rec = inputs.pack_aos(ps, "f32")
    ref = inputs.unpack_aos(rec)
    tol = 1e-5
    pipe = Pipeline(rec, n_c, sched=sched, sub_bits=sub_bits)
    pipe.bin()
    pipe.convert("full")
    it, left = pipe.smoothing_length(tol=tol, max_iter=40)
    assert left == 0 and 2 <= it <= 40
    torch.cuda.synchronize()
    h_rec = pipe.records()["h"].astype(np.float64)
    h_max = _h_max(sph, n_c)
    ho, ito = orc.smoothing_length(ref, n_c=n_c, h_max=h_max, tol=tol, max_iter=40)
    assert np.all(ito <= 40)
    assert np.max(np.abs(h_rec / ho - 1)) < 3 * tol + 1e-5
    assert it >= ito.max() - 1
    # at the root the weighted neighbour number is (4 pi / 3) (gamma_k eta)^3
    pipe.bin()
    pipe.convert("full")
    pipe.density()
    wc = pipe.soa["WCOUNT"].cpu().numpy()
    target = 4.0 * np.pi / 3.0 * (orc.GAMMA_K * orc.ETA) ** 3
    assert np.max(np.abs(wc / target - 1)) < 10 * tol + 1e-4
    # the cells' hmax follows the new h
    cell = pipe.cells.cell.cpu().numpy()
    hs = pipe.soa["H"].cpu().numpy()
    want = np.zeros(n_c ** 3, np.float32)
    np.maximum.at(want, cell, hs)
    assert np.array_equal(pipe.cells.hmax.cpu().numpy(), want)


def test_smoothing_length_capped(sph, orc):
    """Cells too small for the root: h stops at h_max and the particle is
    reported as not converged, as in the oracle."""
    from paper_2512_05516_amd.pipeline import Pipeline
    ps = inputs.small_set(2)
    n_c = 8                 # h_max = 0.125 / gamma_k = 0.068 < the lattice's root 0.077
    ps.h = np.full(ps.n, 0.07)
    rec = inputs.pack_aos(ps, "f32")
    pipe = Pipeline(rec, n_c)
    pipe.bin()
    pipe.convert("full")
    it, left = pipe.smoothing_length(tol=1e-5, max_iter=12)
    assert it == 12 and left == ps.n
    h_max = _h_max(sph, n_c)
    assert np.all(pipe.records()["h"] == np.float32(h_max))
    ho, ito = orc.smoothing_length(inputs.unpack_aos(rec), n_c=n_c, h_max=h_max, tol=1e-5,
                                   max_iter=12, sel=np.arange(64))
    assert np.all(ho == h_max) and np.all(ito == 13)


def test_smoothing_length_full_size_clustered(sph, orc):
    """The 4M clustered set from its analytic h, in a 1.25x roomier cell
    list: the particles that do not converge are exactly those held at
    h_max (roots beyond the cell size, in background voids); a seeded
    sample (background and blob cells) matches the oracle's iteration."""
    from paper_2512_05516_amd.pipeline import Pipeline
    ps = inputs.clustered_k_set(3)
    n_c = int(np.floor(1.0 / (1.25 * orc.GAMMA_K * ps.h.max())))
    rec = inputs.pack_aos(ps, "f32")
    ref = inputs.unpack_aos(rec)
    tol = 1e-4
    pipe = Pipeline(rec, n_c, sched="grid", til=sph.tile(16, 4))
    pipe.bin()
    pipe.convert("full")
    it, left = pipe.smoothing_length(tol=tol, max_iter=30)
    h = pipe.records()["h"].astype(np.float64)
    # the particles left are those whose root lies beyond the cell size
    h_max = _h_max(sph, n_c)
    assert left == np.count_nonzero(h == h_max) and left < 1e-3 * ps.n, left
    rng = np.random.default_rng(21)
    occ = np.diff(pipe.cells.cell_start.cpu().numpy())
    cell_of = np.minimum((ref.x * n_c).astype(int), n_c - 1) @ np.array([1, n_c, n_c * n_c])
    blob = np.nonzero(occ[cell_of] > 400)[0]
    sel = np.unique(np.concatenate([rng.choice(ps.n, 256, replace=False),
                                    rng.choice(blob, 128, replace=False)])).astype(np.int32)
    ho, ito = orc.smoothing_length(ref, n_c=n_c, h_max=h_max, tol=tol, max_iter=30, sel=sel)
    assert np.all((ito <= 30) | (ho == h_max))
    assert np.max(np.abs(h[sel] / ho - 1)) < 3 * tol + 1e-5
    print(f"h iteration on 4M particles: {it} passes, {left} held at h_max")


# ---------------------------------------------------------------------------
# Wendland C2 kernel variant
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("til,sched,sub_bits", [((64, 4), None, 0), ((32, 2), "grid", 1),
                                                ((16, 4), "static", 2)])
def test_wendland_matches_oracle(sph, orc, til, sched, sub_bits):
    """Density and force with the Wendland C2 kernel (gamma_k 1.936492) on a
    clustered set: counts against FP64 brute force, values at the FP32 bar;
    AoS == SoA bit for bit."""
    from paper_2512_05516_amd.pipeline import Pipeline
    prm_o, prm_g = orc.params(kernel="wendland_c2"), sph.params(kernel="wendland_c2")
    assert prm_o.gamma_k == prm_g.gamma_k
    ps = inputs.clustered_set(20000, 9)
    n_c = int(np.floor(1.0 / (prm_o.gamma_k * ps.h.max())))
    pipe = run_gpu(ps, n_c, prm=prm_g, til=sph.tile(*til), sched=sched, sub_bits=sub_bits)
    assert pipe.status() == 0
    got = gpu_fields(pipe)
    ref = inputs.unpack_aos(inputs.pack_aos(ps, "f32"))
    d, f = oracle_step(orc, ref, n_c, prm=prm_o)
    assert_counts(orc, got["nngb"], got["nforce"], d["nngb"], f["nforce"], ref, n_c,
                  gamma_k=prm_o.gamma_k, tag="wendland")
    got["h"] = ref.h
    check_fp32(got, d, f, tag=f"wendland {til} {sched}")
    # the M4 run differs: the kernel choice reaches the loops
    m4 = gpu_fields(run_gpu(ps, n_c, til=sph.tile(*til), sched=sched, sub_bits=sub_bits))
    assert not np.array_equal(m4["rho"], got["rho"])
    if sub_bits == 0:
        pa = Pipeline(inputs.pack_aos(ps, "f32"), n_c, prm=prm_g, til=sph.tile(*til), sched=sched)
        pa.bin()
        pa.density_aos()
        pa.force_aos()
        ra = pa.records()
        for k in ("rho", "wcount", "rho_dh", "f", "P", "c", "nngb", "a", "du", "vsig", "nforce"):
            assert np.array_equal(np.asarray(ra[k]), pipe.records()[k]), k


def test_wendland_smoothing_length(sph, orc):
    """The h iteration with the Wendland kernel reaches the oracle's roots and
    the weighted neighbour number (4 pi / 3)(gamma_k eta)^3 of that kernel."""
    from paper_2512_05516_amd.pipeline import Pipeline
    prm_o, prm_g = orc.params(kernel="wendland_c2"), sph.params(kernel="wendland_c2")
    ps = inputs.small_set(2)
    ps.h = ps.h * np.random.default_rng(4).uniform(0.8, 1.2, ps.n)
    n_c = 4
    rec = inputs.pack_aos(ps, "f32")
    ref = inputs.unpack_aos(rec)
    pipe = Pipeline(rec, n_c, prm=prm_g)
    pipe.bin()
    pipe.convert("full")
    tol = 1e-5
    it, left = pipe.smoothing_length(tol=tol, max_iter=40)
    assert left == 0
    g64 = prm_g.gamma_k
    gk, s = np.float32(g64), np.float32(1.0 / n_c)
    h_max = np.float32(s / gk)
    while (gk * h_max) * (gk * h_max) > s * s or g64 * float(h_max) > 1.0 / n_c:
        h_max = np.nextafter(h_max, np.float32(0))
    ho, _ = orc.smoothing_length(ref, n_c=n_c, h_max=float(h_max), tol=tol, max_iter=40,
                                 prm=prm_o)
    h = pipe.records()["h"].astype(np.float64)
    assert np.max(np.abs(h / ho - 1)) < 3 * tol + 1e-5
    pipe.bin()
    pipe.convert("full")
    pipe.density()
    wc = pipe.soa["WCOUNT"].cpu().numpy()
    target = 4.0 * np.pi / 3.0 * (g64 * orc.ETA) ** 3
    assert np.max(np.abs(wc / target - 1)) < 10 * tol + 1e-4


def test_occupancy_split_launches(sph, orc):
    """A loop run as two launches over occupancy classes (sparse cells with
    one tile, crowded cells with another, sph_worklist_occupancy) gives the
    oracle's results: counts against FP64 brute force, values at the FP32
    bar; the two
    classes partition the cells (every particle's outputs are written)."""
    from paper_2512_05516_amd.pipeline import Pipeline
    ps = inputs.clustered_set(30000, 12, f_blob=0.4)
    n_c = int(np.floor(1.0 / (orc.GAMMA_K * ps.h.max())))
    rec = inputs.pack_aos(ps, "f32")
    ref = inputs.unpack_aos(rec)
    pipe = Pipeline(rec, n_c, sub_bits=1, til=sph.tile(64, 4), til_force=sph.tile(64, 4),
                    sched=("grid", "dynamic"),
                    split={"density": (24, (32, 2), "grid"), "force": (24, (16, 4), "static")})
    occ = None
    pipe.bin()
    occ = np.diff(pipe.cells.cell_start.cpu().numpy())
    assert (occ[occ > 0] < 24).any() and (occ >= 24).any()
    pipe.soa["RHO"].fill_(float("nan"))
    pipe.soa["A_X"].fill_(float("nan"))
    pipe.convert("full")
    pipe.density()
    pipe.force()
    pipe.writeback("full")
    assert pipe.status() == 0
    got = gpu_fields(pipe)
    got["h"] = ref.h
    d, f = oracle_step(orc, ref, n_c)
    assert_counts(orc, got["nngb"], got["nforce"], d["nngb"], f["nforce"], ref, n_c, tag="split")
    check_fp32(got, d, f, tag="split")


@pytest.mark.parametrize("case", ["list64x1", "split32x2", "split64x2/sub2", "f16/split32x2",
                                  "list32x8/sub1"])
def test_merged_items_parity(sph, orc, ragged, case):
    """Work items merging up to four sparse cells along x (one chunk, one
    merged candidate neighbourhood): counts against FP64 brute force and
    values at the FP32 bar on the ragged clustered set (empty cells, partial
    bricks, crowded cells beside sparse ones), over the whole list, over
    the sparse class of a split launch, with sub-cells, and with FP16
    positions anchored at sub-cell centres (against the oracle on the same
    stored values)."""
    from paper_2512_05516_amd.pipeline import Pipeline
    ps, ref, n_c, d, f = ragged
    rec = inputs.pack_aos(ps, "f32")
    prec, sub = None, 0
    if case.startswith("f16"):
        prec = sph.precision("f16", "bf16", "f16", 12, 3, 0, anchor=SUB2)
    if "sub" in case:
        sub = int(case[-1])
    if case.startswith("list"):
        ti, k = (64, 1) if "64x1" in case else (32, 8)
        pipe = Pipeline(rec, n_c, prec=prec, sub_bits=sub, til=sph.tile(ti, k), sched="grid",
                        max_cells=4)
    else:
        ti, k = (32, 2) if "32x2" in case else (64, 2)
        pipe = Pipeline(rec, n_c, prec=prec, sub_bits=sub, til=sph.tile(64, 4),
                        sched=("grid", "dynamic"),
                        split={"density": (32, (ti, k), "grid", 4),
                               "force": (32, (ti, k), "grid", 4)})
    pipe.bin()
    ws = pipe._parts["force"][0][1] if pipe._parts else pipe.work
    items, _, _ = _read_worklist(ws, ps.n, n_c)
    assert (items[:, 0] >> 29).max() > 0                 # some items do merge
    pipe.soa["RHO"].fill_(float("nan"))
    pipe.soa["A_X"].fill_(float("nan"))
    pipe.convert("full")
    pipe.density()
    pipe.force()
    pipe.writeback("full")
    assert pipe.status() == 0
    got = gpu_fields(pipe)
    if prec is None:
        got["h"] = ref.h
        dd, ff, q, tol = d, f, ref, FP32_TOL
    else:
        q = orc.dequantise_set(ref, n_c, "f16", "bf16", "f16", (12, 3, 0), anchor=SUB2)
        got["h"] = q.h
        dd, ff = oracle_step(orc, q, n_c)
        tol = 2e-5
    assert_counts(orc, got["nngb"], got["nforce"], dd["nngb"], ff["nforce"], q, n_c,
                  tag=f"merged/{case}")
    check_fp32(got, dd, ff, tol=tol, tag=f"merged/{case}")


# ---------------------------------------------------------------------------
# keeping the cell list while no particle leaves its cell or sub-cell
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sub_bits,sched", [(0, None), (1, "grid"), (2, "dynamic")])
def test_keep_cells_equals_rebinning(sph, sub_bits, sched):
    """A pipeline that keeps its cell list (and work lists) while the kicks
    count no particle leaving its cell or sub-cell gives records identical
    bit for bit to one that rebins every step: over kick-only steps (no
    drift) the list is kept after the first binning; once particles move
    across cells it is rebuilt, and the moved count equals the number of
    particles whose cell or sub-cell changed."""
    import torch
    from paper_2512_05516_amd.pipeline import Pipeline
    ps = inputs.clustered_set(20000, 5, f_blob=0.4, sigma=0.05)
    n_c = int(np.floor(1.0 / (1.825742 * ps.h.max())))
    rec = inputs.pack_aos(ps, "f32")
    kw = dict(sub_bits=sub_bits, sched=sched)
    keep = Pipeline(rec, n_c, keep_cells=True, **kw)
    full = Pipeline(rec, n_c, **kw)
    rebuilt = []
    for dt_drift in (0.0, 0.0, 0.0, 2e-3, 2e-3, 0.0):
        for p in (keep, full):
            p.soa_step(1e-4, dt_drift)
        torch.cuda.synchronize()
        rebuilt.append(int(keep.cells.rebin[1].item()))
        assert keep.records().tobytes() == full.records().tobytes(), (dt_drift, rebuilt)
    # built once, kept over the kick-only steps, rebuilt after the moves
    assert rebuilt[:4] == [1, 0, 0, 0] and rebuilt[4] == 1, rebuilt
    # the count of the last drifting kick: particles whose cell or sub-cell changed
    x0 = full.records()["x"]
    keep.bin()
    keep.convert("full")
    keep.density()
    keep.force()
    keep.kick_drift(0.0, 5e-3)
    keep.writeback("kick")
    torch.cuda.synchronize()
    x1 = keep.records()["x"]
    R = 1 << sub_bits
    k0 = np.minimum(np.floor(x0 * n_c * R), n_c * R - 1).astype(np.int64)
    k1 = np.minimum(np.floor(x1 * n_c * R), n_c * R - 1).astype(np.int64)
    assert int(keep.cells.rebin[0].item()) == int(np.any(k0 != k1, axis=1).sum()) > 0
    assert keep.status() == 0
