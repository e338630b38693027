"""CPU-only checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments on the host before any device
work (these calls never reach the GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2512_05516_amd import inputs

from helpers import unpack_trunc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sph():
    from paper_2512_05516_amd import sphmi
    if not os.path.exists(sphmi.LIB_PATH):
        from paper_2512_05516_amd import build
        build.build(verbose=False)
    sphmi.lib()
    return sphmi


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "sphmi.h")).read()
    return sorted(set(re.findall(r"^\s*(?:sph_status|int32_t|int64_t|const char \*)\s*(sph_\w+)\(",
                                 txt, re.M)))


def test_exports_every_header_symbol(sph):
    syms = header_symbols()
    assert len(syms) >= 18
    L = sph.lib()
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(sph.EXPORTS)


def test_abi_version_and_tiles(sph):
    assert sph.abi_version() == 11
    assert sph.tile_supported(64, 4)
    assert sph.tile_supported(16, 4) and sph.tile_supported(32, 2)
    assert not sph.tile_supported(48, 3)


def test_position_anchor_validation(sph):
    """pos_anchor must be SPH_ANCHOR_CORNER or SPH_ANCHOR_SUB(0..2) and the
    reserved word 0; anchors at sub-cell centres of depth b >= 1 need the
    ANC codes wherever the offsets are written or read."""
    L = sph.lib()
    cells = _fake_cells(sph)
    lay = sph.layout_from_dtype(inputs.AOS_F32)
    soa = sph.Soa()
    for i in range(len(sph.S_FIELDS)):
        soa.f[i] = 0x4000 + 256 * i
    no_anc = sph.Soa()
    for i in range(len(sph.S_FIELDS)):
        no_anc.f[i] = 0x4000 + 256 * i
    no_anc.f[sph.S["ANC"]] = None
    assert sph.ANCHOR_SUB(2) == 3 and sph.S["ANC"] == len(sph.S_FIELDS) - 1
    for bad in (sph.precision("f16", anchor=4), sph.precision("f16", anchor=-1),
                sph.Precision(sph.F16, sph.F32, sph.F32, 0, 0, 0, 0, 1)):
        assert L.sph_density(C.byref(soa), C.byref(bad), C.byref(cells), C.byref(sph.params()),
                             sph.Tile(0, 0), None, None) == sph.SPH_E_INVALID
    for anchor in (sph.ANCHOR_SUB(1), sph.ANCHOR_SUB(2)):
        p = sph.precision("f16", anchor=anchor)
        for fn in (L.sph_density, L.sph_force):
            assert fn(C.byref(no_anc), C.byref(p), C.byref(cells), C.byref(sph.params()),
                      sph.Tile(0, 0), None, None) == sph.SPH_E_INVALID
            assert "ANC" in sph.last_error()
        assert L.sph_convert(C.c_void_p(0x3000), C.byref(lay), C.byref(cells), 3, C.byref(p),
                             C.byref(no_anc), None) == sph.SPH_E_INVALID
        # the kick view holds no offsets: no codes needed
        assert L.sph_convert(C.c_void_p(0x3000), C.byref(lay), C.byref(_fake_cells(sph, 0)), 2,
                             C.byref(p), C.byref(no_anc), None) == sph.SPH_OK
        buf = np.zeros(1 << 16, np.uint8)
        rec = np.zeros(16, dtype=inputs.AOS_F32)
        assert L.sph_convert_host(C.c_void_p(rec.ctypes.data), C.byref(lay),
                                  C.byref(_fake_cells(sph)), 3, C.byref(p), C.byref(no_anc),
                                  C.c_void_p(buf.ctypes.data), buf.size, 1,
                                  None) == sph.SPH_E_INVALID
    # the cell centre (b = 0) has no codes to store
    p = sph.precision("f16", anchor=sph.ANCHOR_SUB(0))
    assert sph.host_staging_size(1000, 4, "density", p) == \
        sph.host_staging_size(1000, 4, "density", sph.precision("f16"))
    assert sph.host_staging_size(1000, 4, "density", sph.precision("f16", anchor=3)) >= \
        sph.host_staging_size(1000, 4, "density", p) + 1000


def test_workspace_size_validation(sph):
    assert sph.bin_workspace_size(4096, 4) > 4 * 4 * 4096
    assert sph.bin_workspace_size(0, 4) > 0
    with pytest.raises(sph.SphError) as e:
        sph.bin_workspace_size(-1, 4)
    assert e.value.code == sph.SPH_E_INVALID
    with pytest.raises(sph.SphError) as e:
        sph.bin_workspace_size(10, 2)
    assert e.value.code == sph.SPH_E_RANGE
    assert sph.reduce_workspace_size(100) >= 8 * 8
    assert sph.worklist_size(4096, 4, 64) >= 256 + 8 * (64 + 64)
    with pytest.raises(sph.SphError):
        sph.worklist_size(4096, 4, 0)
    p = sph.precision("f16", "bf16", "f16")
    assert sph.host_staging_size(1000, 4, "full", p) > 1000 * (6 + 6 + 6 + 24 + 12 + 4)


def _fake_cells(sph, n=16, n_c=4, lists=True, sub_bits=0, sub=True):
    dummy = C.c_void_p(0x1000) if lists else None
    return sph.Cells(n, n_c, sub_bits, 0, dummy, dummy, dummy, dummy if sub else None, None, None)


def test_host_side_validation(sph):
    L = sph.lib()
    lay = sph.layout_from_dtype(inputs.AOS_F32)
    cells = _fake_cells(sph)
    ws = C.c_void_p(0x2000)
    # NULL layout, bad stride, X not FP64, misaligned field
    assert L.sph_bin(C.c_void_p(0x3000), None, C.byref(cells), ws, 1 << 30, None) == sph.SPH_E_INVALID
    bad = sph.layout_from_dtype(inputs.AOS_F32)
    bad.stride = 12
    assert L.sph_bin(C.c_void_p(0x3000), C.byref(bad), C.byref(cells), ws, 1 << 30, None) == sph.SPH_E_INVALID
    bad = sph.layout_from_dtype(inputs.AOS_F32)
    bad.dtype[sph.A["X"]] = sph.F32
    assert L.sph_bin(C.c_void_p(0x3000), C.byref(bad), C.byref(cells), ws, 1 << 30, None) == sph.SPH_E_INVALID
    assert "X" in sph.last_error()
    bad = sph.layout_from_dtype(inputs.AOS_F32)
    bad.offset[sph.A["M"]] = 126
    assert L.sph_convert(C.c_void_p(0x3000), C.byref(bad), C.byref(cells), 0,
                         C.byref(sph.precision()), C.byref(sph.Soa()), None) == sph.SPH_E_INVALID
    # n_c too small, negative n, workspace too small
    small = _fake_cells(sph, 16, 2)
    assert L.sph_bin(C.c_void_p(0x3000), C.byref(lay), C.byref(small), ws, 1 << 30, None) == sph.SPH_E_RANGE
    neg = _fake_cells(sph, -5, 4)
    assert L.sph_bin(C.c_void_p(0x3000), C.byref(lay), C.byref(neg), ws, 1 << 30, None) == sph.SPH_E_INVALID
    assert L.sph_bin(C.c_void_p(0x3000), C.byref(lay), C.byref(cells), ws, 16, None) == sph.SPH_E_NOMEM
    # missing cell-list pointers
    nolists = _fake_cells(sph, 16, 4, lists=False)
    assert L.sph_bin(C.c_void_p(0x3000), C.byref(lay), C.byref(nolists), ws, 1 << 30, None) == sph.SPH_E_INVALID
    # SoA views with NULL fields, bad precision, bad tile, bad view
    soa = sph.Soa()
    assert L.sph_density(C.byref(soa), C.byref(sph.precision()), C.byref(cells),
                         C.byref(sph.params()), sph.Tile(0, 0), None, None) == sph.SPH_E_INVALID
    for i in range(len(sph.S_FIELDS)):
        soa.f[i] = 0x4000 + 256 * i
    assert L.sph_density(C.byref(soa), C.byref(sph.Precision(7, 1, 1, 0, 0, 0)), C.byref(cells),
                         C.byref(sph.params()), sph.Tile(0, 0), None, None) == sph.SPH_E_INVALID
    assert L.sph_density(C.byref(soa), C.byref(sph.precision()), C.byref(cells),
                         C.byref(sph.params()), sph.Tile(48, 3), None, None) == sph.SPH_E_UNSUPPORTED
    bad_prm = sph.params(gamma_k=float("nan"))
    assert L.sph_force(C.byref(soa), C.byref(sph.precision()), C.byref(cells),
                       C.byref(bad_prm), sph.Tile(0, 0), None, None) == sph.SPH_E_INVALID
    # work list: tile mismatch, missing buffer, too small
    wk = sph.Work(32, 0, C.c_void_p(0x7000), 1 << 30)
    assert L.sph_density(C.byref(soa), C.byref(sph.precision()), C.byref(cells),
                         C.byref(sph.params()), sph.Tile(64, 4), C.byref(wk), None) == sph.SPH_E_INVALID
    wk = sph.Work(64, 0, C.c_void_p(0x7000), 64)
    assert L.sph_density(C.byref(soa), C.byref(sph.precision()), C.byref(cells),
                         C.byref(sph.params()), sph.Tile(64, 4), C.byref(wk), None) == sph.SPH_E_NOMEM
    assert L.sph_worklist(C.byref(cells), C.byref(sph.Work(64, 0, None, 1 << 30)), None) == sph.SPH_E_INVALID
    assert L.sph_worklist(C.byref(cells), C.byref(sph.Work(64, 0, C.c_void_p(0x7000), 64)),
                          None) == sph.SPH_E_NOMEM
    for bad_sched in (-1, 3):
        wk = sph.Work(64, bad_sched, C.c_void_p(0x7000), 1 << 30)
        assert L.sph_density(C.byref(soa), C.byref(sph.precision()), C.byref(cells),
                             C.byref(sph.params()), sph.Tile(64, 4), C.byref(wk),
                             None) == sph.SPH_E_INVALID
        assert "sched" in sph.last_error()
    # merged work items: max_cells in [0, 4], reserved 0
    for mc, rs in ((5, 0), (-1, 0), (4, 1)):
        wk = sph.Work(64, 0, C.c_void_p(0x7000), 1 << 30, mc, rs)
        assert L.sph_worklist(C.byref(cells), C.byref(wk), None) == sph.SPH_E_INVALID
        assert L.sph_density(C.byref(soa), C.byref(sph.precision()), C.byref(cells),
                             C.byref(sph.params()), sph.Tile(64, 4), C.byref(wk),
                             None) == sph.SPH_E_INVALID
    wk = sph.Work(64, 0, C.c_void_p(0x7000), 1 << 44, 2, 0)   # cell ids need n_c^3 < 2^29
    assert L.sph_worklist(C.byref(_fake_cells(sph, 16, 820)), C.byref(wk), None) == sph.SPH_E_RANGE
    # sub-cells: range and the required sub_start table
    assert L.sph_bin(C.c_void_p(0x3000), C.byref(lay), C.byref(_fake_cells(sph, sub_bits=4)), ws,
                     1 << 30, None) == sph.SPH_E_RANGE
    assert L.sph_bin(C.c_void_p(0x3000), C.byref(lay), C.byref(_fake_cells(sph, sub_bits=2, sub=False)),
                     ws, 1 << 30, None) == sph.SPH_E_INVALID
    assert L.sph_bin(C.c_void_p(0x3000), C.byref(lay), C.byref(_fake_cells(sph, n_c=1000, sub_bits=1)),
                     ws, 1 << 36, None) == sph.SPH_E_RANGE
    assert L.sph_convert(C.c_void_p(0x3000), C.byref(lay), C.byref(cells), 9,
                         C.byref(sph.precision()), C.byref(soa), None) == sph.SPH_E_INVALID
    assert L.sph_kick_drift(C.byref(soa), C.byref(cells), float("inf"), 1e-4, None, None) == sph.SPH_E_INVALID
    big_scale = sph.precision("f16", "f16", "f16", scale_m=100)
    assert L.sph_reduce(C.byref(soa), C.byref(big_scale), C.byref(cells), C.c_void_p(0x5000),
                        C.c_void_p(0x6000), 1 << 20, None) == sph.SPH_E_INVALID
    # plain-AoS reductions: the cell list, V/A/DU in the layout, out and a large enough workspace
    out, w6 = C.c_void_p(0x5000), C.c_void_p(0x6000)
    assert L.sph_reduce_aos(C.c_void_p(0x3000), C.byref(lay), C.byref(nolists), out, w6, 1 << 20,
                            None) == sph.SPH_E_INVALID
    bad = sph.layout_from_dtype(inputs.AOS_F32)
    bad.offset[sph.A["A"]] = sph.ABSENT
    assert L.sph_reduce_aos(C.c_void_p(0x3000), C.byref(bad), C.byref(cells), out, w6, 1 << 20,
                            None) == sph.SPH_E_INVALID
    assert L.sph_reduce_aos(C.c_void_p(0x3000), C.byref(lay), C.byref(cells), None, w6, 1 << 20,
                            None) == sph.SPH_E_INVALID
    assert L.sph_reduce_aos(C.c_void_p(0x3000), C.byref(lay), C.byref(cells), out, w6, 16,
                            None) == sph.SPH_E_NOMEM


def test_tuner_host_side(sph):
    L = sph.lib()
    cand = sph.tune_candidates()
    assert len(cand) == 32
    assert len(set(cand)) == 32
    assert {c[2] for c in cand} == {None, "grid", "static", "dynamic"}
    assert all(sph.tile_supported(t, k) for t, k, _ in cand)
    n = C.c_int32()
    assert L.sph_tune_candidates(None, 5, C.byref(n)) == sph.SPH_E_INVALID
    assert L.sph_tune_candidates(None, 0, None) == sph.SPH_E_INVALID
    cells = _fake_cells(sph)
    soa = sph.Soa()
    arr = (sph.TuneEntry * 2)()
    arr[0].tile = sph.Tile(64, 4)
    arr[1].tile = sph.Tile(32, 8)
    best = C.c_int32()
    args = lambda loop, a, nc, reps: L.sph_autotune(loop, C.byref(soa), C.byref(sph.precision()),
                                                  C.byref(cells), C.byref(sph.params()), a, nc,
                                                  reps, None, 0, C.byref(best), None)
    assert args(2, arr, 2, 3) == sph.SPH_E_INVALID
    assert args(0, arr, 0, 3) == sph.SPH_E_INVALID
    assert args(0, arr, 2, 0) == sph.SPH_E_INVALID
    arr[1].sched = 3
    assert args(1, arr, 2, 3) == sph.SPH_E_INVALID
    arr[1].sched = 0
    arr[1].tile = sph.Tile(48, 3)
    assert args(0, arr, 2, 3) == sph.SPH_E_UNSUPPORTED


def test_host_convert_rejects_sub_cells(sph):
    import numpy as np
    L = sph.lib()
    lay = sph.layout_from_dtype(inputs.AOS_F32)
    rec = np.zeros(16, dtype=inputs.AOS_F32)
    cells = _fake_cells(sph, 16, 4, sub_bits=1)
    soa = sph.Soa()
    buf = np.zeros(1 << 16, np.uint8)
    st = L.sph_convert_host(C.c_void_p(rec.ctypes.data), C.byref(lay), C.byref(cells), 3,
                            C.byref(sph.precision()), C.byref(soa), C.c_void_p(buf.ctypes.data),
                            buf.size, 1, None)
    assert st == sph.SPH_E_UNSUPPORTED
    assert "sub_bits" in sph.last_error()


def test_server_host_side(sph):
    L = sph.lib()
    nb = C.c_size_t()
    T0 = sph.Tile(0, 0)
    good = sph.ServerConfig(T0, 4, 256, 64 << 20)
    assert L.sph_server_workspace_size(C.byref(good), C.byref(nb)) == sph.SPH_OK
    assert nb.value >= 64 << 20
    bad = [(sph.ServerConfig(T0, 0, 256, 64 << 20), sph.SPH_E_INVALID),
           (sph.ServerConfig(T0, 9, 256, 64 << 20), sph.SPH_E_INVALID),
           (sph.ServerConfig(T0, 4, 0, 64 << 20), sph.SPH_E_INVALID),
           (sph.ServerConfig(T0, 4, 5000, 64 << 20), sph.SPH_E_INVALID),
           (sph.ServerConfig(T0, 4, 256, 1000), sph.SPH_E_INVALID),
           (sph.ServerConfig(sph.Tile(48, 3), 4, 256, 64 << 20), sph.SPH_E_UNSUPPORTED),
           (sph.ServerConfig(sph.Tile(128, 2), 4, 256, 64 << 20), sph.SPH_E_UNSUPPORTED)]
    for cfg, code in bad:
        assert L.sph_server_workspace_size(C.byref(cfg), C.byref(nb)) == code
    h = C.c_void_p()
    assert L.sph_server_create(C.byref(good), None, None, None, None, None, 0,
                               C.byref(h)) == sph.SPH_E_INVALID
    assert L.sph_task_tile_supported(sph.Tile(64, 4)) == 1
    assert L.sph_task_tile_supported(sph.Tile(16, 16)) == 1
    assert L.sph_task_tile_supported(sph.Tile(128, 2)) == 0
    cells = _fake_cells(sph)
    soa = sph.Soa()
    for i in range(len(sph.S_FIELDS)):
        soa.f[i] = 0x4000 + 256 * i
    args = lambda nd, nf, tile=T0, out=C.c_void_p(0x9000): L.sph_tasks_run(
        C.byref(soa), C.byref(sph.precision()), C.byref(cells), C.byref(sph.params()), tile,
        C.c_void_p(0x7000), 4, C.c_void_p(0x7100), C.c_void_p(0x7200), nd, nf, out, 1 << 20, None)
    assert args(-1, 0) == sph.SPH_E_INVALID
    assert args(1, 0, tile=sph.Tile(128, 2)) == sph.SPH_E_UNSUPPORTED
    assert args(1, 1, out=None) == sph.SPH_E_INVALID
    assert args(1, 1, out=C.c_void_p(0x9004)) == sph.SPH_E_INVALID
    assert args(0, 0) == sph.SPH_OK                    # nothing to launch
    t0 = L.sph_now_ns()
    assert L.sph_now_ns() >= t0 > 0


def test_task_stream_generator():
    from paper_2512_05516_amd import serve
    n_c = 5
    occ = np.random.default_rng(1).integers(0, 900, n_c ** 3)
    start = np.concatenate([[0], np.cumsum(occ)])
    tasks = serve.make_tasks(start, n_c, 2000, seed=3)
    assert tasks.shape == (2000, 5)
    size = tasks[:, 4] - tasks[:, 3]
    assert size.min() >= 16 // 2 and size.max() <= 512
    assert np.all(tasks[:, 3] >= start[tasks[:, 1]]) and np.all(tasks[:, 4] <= start[tasks[:, 1] + 1])
    assert np.all(occ[tasks[:, 2]] >= 16) and np.all(occ[tasks[:, 1]] >= 16)
    c = lambda v: np.stack([v % n_c, (v // n_c) % n_c, v // n_c ** 2], 1)
    d = (c(tasks[:, 2]) - c(tasks[:, 1])) % n_c
    assert np.all((d == 0) | (d == 1) | (d == n_c - 1))
    assert 0.4 < tasks[:, 0].mean() < 0.6
    arr = serve.poisson_arrivals(20000, 1e4, 0, seed=2)
    gaps = np.diff(arr) * 1e-9
    assert abs(gaps.mean() - 1e-4) < 5e-6 and np.all(gaps >= 0)
    req, offs = serve.requests(tasks, np.zeros(2000, np.int64), out_ptr=1 << 20)
    assert req["out"][1] - req["out"][0] == 32 * size[0]


def test_truncated_storage_host_side(sph):
    import math
    for n in (0, 1, 255, 256, 1000):
        assert sph.storage_bytes(n, sph.F32) == 4 * n
        assert sph.storage_bytes(n, sph.F16) == 2 * n
        for T in (9, 16, 20, 32):
            assert sph.storage_bytes(n, sph.DT[f"t{T}"]) == (math.ceil(n / 256) * 8 * T + 2) * 4
    with pytest.raises(sph.SphError):
        sph.storage_bytes(10, sph.TRUNC + 33)
    with pytest.raises(sph.SphError):
        sph.storage_bytes(10, sph.F64)
    # host unpacking of a bitstream packed here value by value
    rng = np.random.default_rng(3)
    for T in (9, 13, 16, 17, 24, 31, 32):
        n = 700
        codes = rng.integers(0, 1 << T, n, dtype=np.uint64)
        bits = np.zeros(((n * T + 31) // 32 + 2) * 32, np.uint8)
        for k, c in enumerate(codes):
            for b in range(T):
                bits[k * T + b] = (int(c) >> b) & 1
        words = np.packbits(bits.reshape(-1, 8)[:, ::-1]).view(np.uint32)
        got = unpack_trunc(words, T, n)
        want = ((codes << np.uint64(32 - T)).astype(np.uint32).view(np.float32) if T > 16 else
                (codes << np.uint64(16 - T)).astype(np.uint16).view(np.float16).astype(np.float32))
        assert np.array_equal(got.view(np.uint32), np.asarray(want, np.float32).view(np.uint32)), T
    # truncated storage is written by sph_convert only
    L = sph.lib()
    lay = sph.layout_from_dtype(inputs.AOS_F32)
    rec = np.zeros(16, dtype=inputs.AOS_F32)
    buf = np.zeros(1 << 16, np.uint8)
    st = L.sph_convert_host(C.c_void_p(rec.ctypes.data), C.byref(lay), C.byref(_fake_cells(sph)),
                            3, C.byref(sph.precision("t20", "f32", "f32")), C.byref(sph.Soa()),
                            C.c_void_p(buf.ctypes.data), buf.size, 1, None)
    assert st == sph.SPH_E_UNSUPPORTED
    big = sph.layout_from_dtype(inputs.AOS_F32)
    big.stride = 256
    soa = sph.Soa()
    for i in range(len(sph.S_FIELDS)):
        soa.f[i] = 0x4000 + 256 * i
    assert L.sph_convert(C.c_void_p(0x3000), C.byref(big), C.byref(_fake_cells(sph)), 3,
                         C.byref(sph.precision("t20", "t20", "t20")), C.byref(soa),
                         None) == sph.SPH_E_UNSUPPORTED


def test_layout_from_numpy(sph):
    lay = sph.layout_from_dtype(inputs.AOS_F32)
    assert lay.stride == 128
    assert lay.offset[sph.A["X"]] == 8 and lay.dtype[sph.A["X"]] == sph.F64
    assert lay.offset[sph.A["V"]] == 32 and lay.dtype[sph.A["V"]] == sph.F32
    lay = sph.layout_from_dtype(inputs.AOS_F64)
    assert lay.stride == 200 and lay.dtype[sph.A["RHO"]] == sph.F64
    assert lay.dtype[sph.A["NNGB"]] == sph.I32


def test_inputs_recipe():
    ps = inputs.small_set(1)
    assert ps.n == 4096
    assert np.all((ps.x >= 0) & (ps.x < 1))
    assert np.all(ps.m == 2.0 ** -12)
    assert np.allclose(ps.h, inputs.ETA / 16)
    # the jitter keeps every particle inside its lattice block of 4^3 sites
    b = np.floor(ps.x * 4).astype(int)
    site = np.floor(ps.x * 16).astype(int)
    assert np.array_equal(site // 4, b)
    # 'blocked' order: consecutive runs of 64 share one block
    pb = inputs.lattice_set(16, 1, order="blocked")
    blk = np.floor(pb.x * 4).astype(int)
    key = blk[:, 0] + 4 * (blk[:, 1] + 4 * blk[:, 2])
    assert np.all(key.reshape(-1, 64) == key.reshape(-1, 64)[:, :1])


def test_host_binning_and_streaming_checks(sph, orc):
    """sph_bin_host follows the binning definition (numpy floor + stable
    lexsort, per-cell largest h); the streaming gather and writeback reject
    bad views, short staging and out-of-range cell lists on the host."""
    ps = inputs.small_set(5)
    rec = inputs.pack_aos(ps, "f32")
    lay = sph.layout_from_dtype(rec.dtype)
    n_c = 4
    start, perm, cell, hmax = sph.bin_host(rec, lay, n_c, nthreads=3)
    x = ps.x - np.floor(ps.x)
    c3 = np.minimum(np.floor(x * n_c).astype(np.int64), n_c - 1)
    ref_cell = c3[:, 0] + n_c * (c3[:, 1] + n_c * c3[:, 2])
    ref_perm = np.lexsort((np.arange(ps.n), ref_cell))
    assert np.array_equal(perm, ref_perm)
    assert np.array_equal(cell, ref_cell[ref_perm])
    assert np.array_equal(start, np.searchsorted(ref_cell[ref_perm], np.arange(n_c ** 3 + 1)))
    hm = np.zeros(n_c ** 3, np.float32)
    np.maximum.at(hm, ref_cell, rec["h"].astype(np.float32))
    assert np.array_equal(hmax, hm)
    # more threads than one give the same list (stable by input index)
    big = np.concatenate([rec] * 2)
    a = sph.bin_host(big, lay, n_c, nthreads=1)
    b = sph.bin_host(big, lay, n_c, nthreads=7)
    assert all(np.array_equal(u, v) for u, v in zip(a, b))

    L = sph.lib()
    soa = sph.Soa()
    prec = sph.precision()
    buf = np.zeros(1 << 20, np.uint8)
    bad = perm.copy()
    bad[3] = ps.n
    args = lambda view, p_, nbytes: L.sph_gather_host(
        C.c_void_p(rec.ctypes.data), C.byref(lay), ps.n, n_c, C.c_void_p(p_.ctypes.data),
        C.c_void_p(cell.ctypes.data), view, C.byref(prec), C.byref(soa),
        C.c_void_p(buf.ctypes.data), nbytes, 1, None)
    assert args(9, perm, buf.size) == sph.SPH_E_INVALID            # unknown view
    assert args(4, perm, buf.size) == sph.SPH_E_INVALID            # soa fields are NULL
    for f in range(len(sph.S_FIELDS)):                             # any non-NULL pointer
        soa.f[f] = buf.ctypes.data
    assert args(4, bad, buf.size) == sph.SPH_E_RANGE
    assert args(4, perm, 16) == sph.SPH_E_NOMEM
    out = C.c_size_t()
    assert L.sph_writeback_host_size(ps.n, 4, C.byref(out)) == sph.SPH_E_INVALID
    assert L.sph_writeback_host_size(ps.n, 2, C.byref(out)) == sph.SPH_OK
    assert out.value >= ps.n * (3 * 8 + 4 * 4)
    st = L.sph_writeback_host(C.byref(soa), ps.n, C.c_void_p(bad.ctypes.data), 2,
                              C.c_void_p(rec.ctypes.data), C.byref(lay),
                              C.c_void_p(buf.ctypes.data), buf.size, 1, None)
    assert st == sph.SPH_E_RANGE


def test_leapfrog_entry_points_host_side(sph):
    """sph_predict / sph_step_totals reject bad arguments before any launch."""
    L = sph.lib()
    lay = sph.layout_from_dtype(inputs.AOS_F32)
    cells = _fake_cells(sph)
    soa = sph.Soa()
    for f in range(len(sph.S_FIELDS)):
        soa.f[f] = 0x4000
    prec = sph.precision()
    aos = C.c_void_p(0x8000)
    pred = lambda s, p, l, dth: L.sph_predict(s, C.byref(p), C.byref(cells), aos, l, dth, None)
    assert pred(None, prec, C.byref(lay), 1e-3) == sph.SPH_E_INVALID
    assert pred(C.byref(soa), sph.precision("t20", "t20", "t20"), C.byref(lay),
                1e-3) == sph.SPH_E_UNSUPPORTED
    assert pred(C.byref(soa), prec, C.byref(lay), float("nan")) == sph.SPH_E_INVALID
    no_a = sph.layout_from_dtype(inputs.AOS_F32)
    no_a.offset[sph.A["A"]] = sph.ABSENT
    assert pred(C.byref(soa), prec, C.byref(no_a), 1e-3) == sph.SPH_E_INVALID
    out = C.c_void_p(0x9000)
    tot = lambda c, ws, nb: L.sph_step_totals(C.byref(soa), C.byref(prec), C.byref(cells),
                                              C.byref(sph.params()), c, out, ws, nb, None)
    need = sph.reduce_workspace_size(16)
    assert tot(0.0, C.c_void_p(0xa000), need) == sph.SPH_E_INVALID
    assert tot(0.1, None, need) == sph.SPH_E_INVALID
    assert tot(0.1, C.c_void_p(0xa000), need - 8) == sph.SPH_E_NOMEM


def test_worklist_occupancy_host_side(sph):
    """sph_worklist_occupancy rejects empty or negative occupancy ranges and
    bad work buffers before any launch."""
    L = sph.lib()
    cells = _fake_cells(sph, 16, 4)
    need = sph.worklist_size(16, 4, 64)
    work = sph.Work(64, 0, C.c_void_p(0x2000), need)
    assert L.sph_worklist_occupancy(C.byref(cells), C.byref(work), 5, 5, None) == sph.SPH_E_INVALID
    assert L.sph_worklist_occupancy(C.byref(cells), C.byref(work), -1, 8, None) == sph.SPH_E_INVALID
    small = sph.Work(64, 0, C.c_void_p(0x2000), need - 1)
    assert L.sph_worklist_occupancy(C.byref(cells), C.byref(small), 0, 8, None) == sph.SPH_E_NOMEM
    bad = sph.Work(64, 7, C.c_void_p(0x2000), need)
    assert L.sph_worklist_occupancy(C.byref(cells), C.byref(bad), 0, 8, None) == sph.SPH_E_INVALID


def _brick_cell(j, n_c, b=4):
    """The closed form the launches use to map a position j in brick order
    to a cell id (mixed radix over z-layers, rows and bricks of b cells,
    thinner at the upper edge)."""
    nb = (n_c + b - 1) // b
    last = n_c - b * (nb - 1)
    layer = b * n_c * n_c
    bz = min(j // layer, nb - 1)
    r = j - bz * layer
    tz = last if bz == nb - 1 else b
    row = tz * b * n_c
    by = min(r // row, nb - 1)
    r -= by * row
    ty = last if by == nb - 1 else b
    col = tz * ty * b
    bx = min(r // col, nb - 1)
    r -= bx * col
    tx = last if bx == nb - 1 else b
    lx, ly, lz = r % tx, (r // tx) % ty, r // (tx * ty)
    return (b * bx + lx) + n_c * ((b * by + ly) + n_c * (b * bz + lz))


@pytest.mark.parametrize("n_c", [3, 4, 5, 7, 8, 13, 32, 33, 44])
def test_brick_order_closed_form(n_c):
    """The closed-form brick order equals the direct enumeration of bricks
    and is a permutation of the cells (every n_c mod 4, including n_c < 4)."""
    from helpers import brick_order
    want = brick_order(n_c)
    got = np.array([_brick_cell(j, n_c) for j in range(n_c ** 3)])
    assert np.array_equal(got, want)
    assert np.array_equal(np.sort(got), np.arange(n_c ** 3))
