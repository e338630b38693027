"""ctypes binding of libsphmi (include/sphmi.h): argument marshalling only.

Every step of the hot path runs in the HIP library; this module turns torch
device tensors into raw pointers and ABI structs, calls the entry point of
the same name and raises SphError on a non-zero status. PyTorch provides
device memory and streams and nothing else. There is no fallback: if the
library is missing, ``lib()`` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsphmi.so")

# --- constants mirrored from include/sphmi.h --------------------------------
SPH_OK, SPH_E_INVALID, SPH_E_RANGE, SPH_E_NOMEM, SPH_E_HIP, SPH_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
FLAG_BAD_POSITION, FLAG_H_TOO_LARGE = 1, 2
F64, F32, F16, BF16, I32 = 0, 1, 2, 3, 4
TRUNC = 0x100
DT = {"f64": F64, "f32": F32, "f16": F16, "bf16": BF16, "i32": I32}
# truncate_mantissa storage of T bits in total: "t9" ... "t32"
DT.update({f"t{T}": TRUNC + T for T in range(9, 33)})
ABSENT = 0xFFFFFFFF

A_FIELDS = ["X", "V", "A", "M", "H", "U", "RHO", "P", "C", "DU", "RHO_DH", "WCOUNT", "F",
            "VSIG", "NNGB", "NFORCE", "CELL"]
A = {name: i for i, name in enumerate(A_FIELDS)}

S_FIELDS = ["OFF_X", "OFF_Y", "OFF_Z", "VQ_X", "VQ_Y", "VQ_Z", "M", "H", "U",
            "X_X", "X_Y", "X_Z", "V_X", "V_Y", "V_Z", "UK",
            "RHO", "WCOUNT", "RHO_DH", "F", "P", "C", "NNGB",
            "A_X", "A_Y", "A_Z", "DU", "VSIG", "NFORCE", "ANC"]
S = {name: i for i, name in enumerate(S_FIELDS)}

VIEW_DENSITY, VIEW_FORCE, VIEW_KICK, VIEW_FULL = 0, 1, 2, 3
VIEW_FORCE_IN, VIEW_KICK_IN = 4, 5
VIEWS = {"density": VIEW_DENSITY, "force": VIEW_FORCE, "kick": VIEW_KICK, "full": VIEW_FULL,
         "force_in": VIEW_FORCE_IN, "kick_in": VIEW_KICK_IN}


class SphError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sph status {code}: {msg}")
        self.code = code


class AosLayout(C.Structure):
    _fields_ = [("stride", C.c_uint32), ("offset", C.c_uint32 * len(A_FIELDS)),
                ("dtype", C.c_int32 * len(A_FIELDS))]


class Cells(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_c", C.c_int32), ("sub_bits", C.c_int32),
                ("reserved", C.c_int32), ("cell_start", C.c_void_p), ("perm", C.c_void_p),
                ("cell", C.c_void_p), ("sub_start", C.c_void_p), ("hmax", C.c_void_p),
                ("status", C.c_void_p), ("tally", C.c_void_p), ("rebin", C.c_void_p)]


class Work(C.Structure):
    _fields_ = [("ti", C.c_int32), ("sched", C.c_int32), ("buf", C.c_void_p),
                ("bytes", C.c_size_t), ("max_cells", C.c_int32), ("reserved", C.c_int32)]


class Soa(C.Structure):
    _fields_ = [("f", C.c_void_p * len(S_FIELDS))]


ANCHOR_CORNER = 0


def ANCHOR_SUB(b: int) -> int:
    """Position anchor at the centre of the sub-cell of side 1/(n_c 2^b)."""
    return 1 + int(b)


class Precision(C.Structure):
    _fields_ = [("pos", C.c_int32), ("vel", C.c_int32), ("mhu", C.c_int32),
                ("scale_m", C.c_int32), ("scale_h", C.c_int32), ("scale_u", C.c_int32),
                ("pos_anchor", C.c_int32), ("reserved", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("gamma_k", C.c_double), ("gamma", C.c_double), ("alpha", C.c_double),
                ("beta", C.c_double), ("gradh", C.c_int32), ("kernel", C.c_int32)]


KERNEL_M4, KERNEL_WENDLAND_C2 = 0, 1
KERNELS = {"m4": KERNEL_M4, "wendland_c2": KERNEL_WENDLAND_C2}
GAMMA_K = {KERNEL_M4: 1.825742, KERNEL_WENDLAND_C2: 1.936492}   # H / h per kernel


class Tile(C.Structure):
    _fields_ = [("ti", C.c_int32), ("k", C.c_int32)]


class ServerConfig(C.Structure):
    _fields_ = [("tile", Tile), ("streams", C.c_int32), ("max_batch", C.c_int32),
                ("pool_bytes", C.c_size_t)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("done", C.c_int64), ("batches", C.c_int64),
                ("admission_waits", C.c_int64), ("max_inflight", C.c_int32),
                ("reserved", C.c_int32), ("pool_high_water", C.c_int64)]


class TuneEntry(C.Structure):
    _fields_ = [("tile", Tile), ("sched", C.c_int32), ("ms", C.c_float)]


EXPORTS = [
    "sph_abi_version", "sph_last_error", "sph_tile_supported", "sph_bin_workspace_size",
    "sph_bin", "sph_convert", "sph_host_staging_size", "sph_convert_host", "sph_writeback",
    "sph_density", "sph_force", "sph_kick_drift", "sph_reduce_workspace_size", "sph_reduce",
    "sph_density_aos", "sph_force_aos", "sph_kick_drift_aos", "sph_sync", "sph_worklist_size",
    "sph_worklist", "sph_tune_candidates", "sph_autotune", "sph_task_tile_supported",
    "sph_tasks_run", "sph_now_ns", "sph_server_workspace_size", "sph_server_create",
    "sph_server_submit", "sph_server_poll", "sph_server_get_stats", "sph_server_drain",
    "sph_server_destroy", "sph_storage_bytes", "sph_smoothing_length_workspace_size",
    "sph_smoothing_length", "sph_bin_host", "sph_gather_host", "sph_writeback_host_size",
    "sph_writeback_host", "sph_predict", "sph_step_totals", "sph_worklist_occupancy",
    "sph_reduce_static", "sph_hbm_probe", "sph_reduce_aos",
]

_lib = None


def lib():
    """Load libsphmi.so (built by ``python -m paper_2512_05516_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2512_05516_amd.build` (no fallback path exists)")
    L = C.CDLL(LIB_PATH)
    vp, i32, sz, st = C.c_void_p, C.c_int32, C.c_size_t, C.c_int32
    P = C.POINTER
    L.sph_abi_version.restype = i32
    L.sph_last_error.restype = C.c_char_p
    L.sph_tile_supported.argtypes = [Tile]
    L.sph_tile_supported.restype = i32
    L.sph_bin_workspace_size.argtypes = [i32, i32, P(sz)]
    L.sph_bin.argtypes = [vp, P(AosLayout), P(Cells), vp, sz, vp]
    L.sph_convert.argtypes = [vp, P(AosLayout), P(Cells), i32, P(Precision), P(Soa), vp]
    L.sph_host_staging_size.argtypes = [i32, i32, i32, P(Precision), P(sz)]
    L.sph_convert_host.argtypes = [vp, P(AosLayout), P(Cells), i32, P(Precision), P(Soa), vp, sz,
                                   i32, vp]
    L.sph_writeback.argtypes = [P(Soa), P(Cells), i32, vp, P(AosLayout), vp]
    L.sph_bin_host.argtypes = [vp, P(AosLayout), i32, i32, vp, vp, vp, vp, i32]
    L.sph_gather_host.argtypes = [vp, P(AosLayout), i32, i32, vp, vp, i32, P(Precision), P(Soa),
                                  vp, sz, i32, vp]
    L.sph_writeback_host_size.argtypes = [i32, i32, P(sz)]
    L.sph_predict.argtypes = [P(Soa), P(Precision), P(Cells), vp, P(AosLayout), C.c_double, vp]
    L.sph_step_totals.argtypes = [P(Soa), P(Precision), P(Cells), P(Params), C.c_double, vp, vp,
                                  sz, vp]
    L.sph_writeback_host.argtypes = [P(Soa), i32, vp, i32, vp, P(AosLayout), vp, sz, i32, vp]
    L.sph_worklist_size.argtypes = [i32, i32, i32, P(sz)]
    L.sph_worklist.argtypes = [P(Cells), P(Work), vp]
    L.sph_worklist_occupancy.argtypes = [P(Cells), P(Work), i32, i32, vp]
    L.sph_density.argtypes = [P(Soa), P(Precision), P(Cells), P(Params), Tile, P(Work), vp]
    L.sph_force.argtypes = [P(Soa), P(Precision), P(Cells), P(Params), Tile, P(Work), vp]
    L.sph_kick_drift.argtypes = [P(Soa), P(Cells), C.c_double, C.c_double, vp, vp]
    L.sph_reduce_workspace_size.argtypes = [i32, P(sz)]
    L.sph_reduce.argtypes = [P(Soa), P(Precision), P(Cells), vp, vp, sz, vp]
    L.sph_reduce_static.argtypes = [P(Soa), P(Precision), P(Cells), vp, vp]
    L.sph_hbm_probe.argtypes = [i32, vp, vp, sz, vp]
    L.sph_reduce_aos.argtypes = [vp, P(AosLayout), P(Cells), vp, vp, sz, vp]
    L.sph_density_aos.argtypes = [vp, P(AosLayout), P(Cells), P(Params), Tile, P(Work), vp]
    L.sph_force_aos.argtypes = [vp, P(AosLayout), P(Cells), P(Params), Tile, P(Work), vp]
    L.sph_kick_drift_aos.argtypes = [vp, P(AosLayout), P(Cells), C.c_double, C.c_double, vp, vp]
    L.sph_sync.argtypes = [vp]
    L.sph_tune_candidates.argtypes = [P(TuneEntry), i32, P(i32)]
    L.sph_task_tile_supported.argtypes = [Tile]
    L.sph_tasks_run.argtypes = [P(Soa), P(Precision), P(Cells), P(Params), Tile, vp, i32, vp, vp,
                                i32, i32, vp, i32, vp]
    L.sph_now_ns.argtypes = []
    L.sph_storage_bytes.argtypes = [i32, i32, P(sz)]
    L.sph_smoothing_length_workspace_size.argtypes = [i32, P(sz)]
    L.sph_smoothing_length.argtypes = [P(Soa), P(Precision), P(Cells), P(Params), C.c_double,
                                       C.c_double, i32, Tile, P(Work), vp, sz, vp,
                                       P(AosLayout), P(i32), P(i32), vp]
    L.sph_server_workspace_size.argtypes = [P(ServerConfig), P(sz)]
    L.sph_server_create.argtypes = [P(ServerConfig), P(Soa), P(Precision), P(Cells), P(Params),
                                    vp, sz, P(vp)]
    L.sph_server_submit.argtypes = [vp, vp, i32, P(C.c_int64)]
    L.sph_server_poll.argtypes = [vp, vp, i32, P(i32), i32]
    L.sph_server_get_stats.argtypes = [vp, P(ServerStats)]
    L.sph_server_drain.argtypes = [vp, i32]
    L.sph_server_destroy.argtypes = [vp]
    L.sph_autotune.argtypes = [i32, P(Soa), P(Precision), P(Cells), P(Params), P(TuneEntry), i32,
                               i32, vp, sz, P(i32), vp]
    for name in EXPORTS[3:]:
        getattr(L, name).restype = st
    L.sph_task_tile_supported.restype = i32
    L.sph_now_ns.restype = C.c_int64
    _lib = L
    return L


def _check(code):
    if code != SPH_OK:
        raise SphError(code, lib().sph_last_error().decode())


def last_error() -> str:
    return lib().sph_last_error().decode()


# --- struct builders ----------------------------------------------------------
_NUMPY_FIELD = {"x": "X", "v": "V", "a": "A", "m": "M", "h": "H", "u": "U", "rho": "RHO",
                "P": "P", "c": "C", "du": "DU", "rho_dh": "RHO_DH", "wcount": "WCOUNT",
                "f": "F", "vsig": "VSIG", "nngb": "NNGB", "nforce": "NFORCE", "cell": "CELL"}


def layout_from_dtype(dt: np.dtype) -> AosLayout:
    """AoS layout struct from a numpy structured record dtype."""
    lay = AosLayout()
    lay.stride = dt.itemsize
    for i in range(len(A_FIELDS)):
        lay.offset[i] = ABSENT
        lay.dtype[i] = 0
    for name, fid in _NUMPY_FIELD.items():
        if name not in dt.names:
            continue
        fdt, off = dt.fields[name][:2]
        base = fdt.base if fdt.shape else fdt
        code = {np.dtype("<f8"): F64, np.dtype("<f4"): F32, np.dtype("<i4"): I32}[np.dtype(base)]
        lay.offset[A[fid]] = off
        lay.dtype[A[fid]] = code
    return lay


def precision(pos="f32", vel="f32", mhu="f32", scale_m=0, scale_h=0, scale_u=0,
              anchor=ANCHOR_CORNER) -> Precision:
    return Precision(DT[pos], DT[vel], DT[mhu], scale_m, scale_h, scale_u, int(anchor), 0)


def params(gamma_k=None, gamma=5.0 / 3.0, alpha=0.8, beta=3.0, gradh=True,
           kernel="m4") -> Params:
    k = KERNELS.get(kernel, kernel)
    return Params(GAMMA_K[k] if gamma_k is None else gamma_k, gamma, alpha, beta,
                  1 if gradh else 0, k)


def tile(ti=0, k=0) -> Tile:
    return Tile(ti, k)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# --- device buffers (torch allocations) --------------------------------------
_TORCH_DT = {F32: "float32", F16: "float16", BF16: "bfloat16"}


class DeviceCells:
    """Cell list arrays on the device: cell_start[C+1], perm[n], cell[n],
    sub_start[C 8^sub_bits + 1] (sub_bits > 0), hmax[C], status[1], and
    with tally=True the pair loops' work counters tally[2] (int64)."""

    def __init__(self, n: int, n_c: int, device="cuda", sub_bits: int = 0, tally=False,
                 rebin=False):
        import torch
        self.n, self.n_c, self.sub_bits = int(n), int(n_c), int(sub_bits)
        C_ = self.n_c ** 3
        self.cell_start = torch.zeros(C_ + 1, dtype=torch.int32, device=device)
        self.perm = torch.zeros(max(self.n, 1), dtype=torch.int32, device=device)
        self.cell = torch.zeros(max(self.n, 1), dtype=torch.int32, device=device)
        self.sub_start = (torch.zeros(C_ * 8 ** self.sub_bits + 1, dtype=torch.int32, device=device)
                          if self.sub_bits else None)
        self.hmax = torch.zeros(C_, dtype=torch.float32, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        self.tally = torch.zeros(2, dtype=torch.int64, device=device) if tally else None
        # rebin = [moved since the list was built, rebuilt by the last bin]:
        # starts "stale" so the first bin builds the list
        self.rebin = torch.ones(2, dtype=torch.int32, device=device) if rebin else None
        self._s = Cells(self.n, self.n_c, self.sub_bits, 0, self.cell_start.data_ptr(),
                        self.perm.data_ptr(), self.cell.data_ptr(),
                        self.sub_start.data_ptr() if self.sub_start is not None else None,
                        self.hmax.data_ptr(), self.status.data_ptr(),
                        self.tally.data_ptr() if tally else None,
                        self.rebin.data_ptr() if rebin else None)

    def invalidate(self):
        """Mark the cell list stale (records changed other than by a kick):
        the next bin rebuilds it, and work lists are rebuilt now."""
        if self.rebin is not None:
            self.rebin.fill_(1)

    @property
    def struct(self) -> Cells:
        return self._s


SCHEDS = {"grid": 0, "static": 1, "dynamic": 2}


class DeviceWork:
    """Work-list buffer of the pair kernels for tile size ti, taken with
    schedule `sched` ("grid", "static" or "dynamic"); with_sched() gives a
    view of the same list under another schedule. max_cells > 1 lets an
    item hold the slots of up to that many (<= 4) sparse cells along x."""

    def __init__(self, n: int, n_c: int, ti: int, device="cuda", sched="grid", _buf=None,
                 max_cells: int = 1):
        import torch
        nbytes = worklist_size(n, n_c, ti)
        self.n, self.n_c, self.ti, self.sched = n, n_c, int(ti), sched
        self.max_cells = int(max_cells)
        self.buf = (_buf if _buf is not None else
                    torch.empty(nbytes, dtype=torch.uint8, device=device))
        self._s = Work(int(ti), SCHEDS[sched], self.buf.data_ptr(), nbytes, self.max_cells, 0)

    def with_sched(self, sched: str) -> "DeviceWork":
        return DeviceWork(self.n, self.n_c, self.ti, sched=sched, _buf=self.buf,
                          max_cells=self.max_cells)

    @property
    def struct(self) -> Work:
        return self._s


def storage_bytes(n: int, dtype: int) -> int:
    out = C.c_size_t()
    _check(lib().sph_storage_bytes(int(n), int(dtype), C.byref(out)))
    return out.value


class DeviceSoa:
    """SoA arrays (sorted-slot order) for the given storage precision
    (truncated formats: packed 32-bit words, value k at bits [kT, kT + T))."""

    def __init__(self, n: int, prec: Precision, device="cuda", fields=None):
        import torch
        self.n = int(n)
        self.prec = prec
        nn = max(self.n, 1)
        dt = lambda code: getattr(torch, _TORCH_DT.get(code, "int32"))
        spec = {}
        for a in ("X", "Y", "Z"):
            spec["OFF_" + a] = dt(prec.pos)
            spec["VQ_" + a] = dt(prec.vel)
            spec["X_" + a] = torch.float64
            spec["V_" + a] = torch.float32
            spec["A_" + a] = torch.float32
        for k in ("M", "H", "U"):
            spec[k] = dt(prec.mhu)
        for k in ("UK", "RHO", "WCOUNT", "RHO_DH", "F", "P", "C", "DU", "VSIG"):
            spec[k] = torch.float32
        spec["NNGB"] = torch.int32
        spec["NFORCE"] = torch.int32
        spec["ANC"] = torch.uint8
        want = fields if fields is not None else S_FIELDS
        code = {}
        for a in ("X", "Y", "Z"):
            code["OFF_" + a], code["VQ_" + a] = prec.pos, prec.vel
        for k in ("M", "H", "U"):
            code[k] = prec.mhu
        self.packed = {k: c - TRUNC for k, c in code.items() if c >= TRUNC}
        self.t = {}
        for k in want:
            if k in self.packed:
                words = storage_bytes(nn, code[k]) // 4
                self.t[k] = torch.zeros(words, dtype=torch.int32, device=device)
            else:
                self.t[k] = torch.zeros(nn, dtype=spec[k], device=device)
        self._s = Soa()
        for k, v in self.t.items():
            self._s.f[S[k]] = v.data_ptr()

    def __getitem__(self, k):
        return self.t[k] if k in self.packed else self.t[k][: self.n]

    @property
    def struct(self) -> Soa:
        return self._s


# --- entry points ------------------------------------------------------------
def abi_version() -> int:
    return lib().sph_abi_version()


def tile_supported(ti, k) -> bool:
    return bool(lib().sph_tile_supported(Tile(ti, k)))


def bin_workspace_size(n, n_c) -> int:
    out = C.c_size_t()
    _check(lib().sph_bin_workspace_size(n, n_c, C.byref(out)))
    return out.value


def reduce_workspace_size(n) -> int:
    out = C.c_size_t()
    _check(lib().sph_reduce_workspace_size(n, C.byref(out)))
    return out.value


def worklist_size(n, n_c, ti) -> int:
    out = C.c_size_t()
    _check(lib().sph_worklist_size(n, n_c, ti, C.byref(out)))
    return out.value


def worklist(cells: DeviceCells, work: DeviceWork, stream=None, occupancy=None):
    """Build `work` from the cell list; occupancy=(lo, hi) keeps only the
    cells holding lo <= count < hi particles."""
    if occupancy is None:
        _check(lib().sph_worklist(C.byref(cells.struct), C.byref(work.struct), _stream(stream)))
    else:
        lo, hi = occupancy
        _check(lib().sph_worklist_occupancy(C.byref(cells.struct), C.byref(work.struct), int(lo),
                                            int(min(hi, 2 ** 31 - 1)), _stream(stream)))


def _wk(work):
    return C.byref(work.struct) if work is not None else None


def host_staging_size(n, n_c, view, prec) -> int:
    out = C.c_size_t()
    _check(lib().sph_host_staging_size(n, n_c, VIEWS.get(view, view), C.byref(prec), C.byref(out)))
    return out.value


def bin(aos, layout, cells: DeviceCells, workspace, stream=None):
    _check(lib().sph_bin(_ptr(aos), C.byref(layout), C.byref(cells.struct), _ptr(workspace),
                         workspace.numel() * workspace.element_size(), _stream(stream)))


def convert(aos, layout, cells: DeviceCells, view, soa: DeviceSoa, stream=None):
    _check(lib().sph_convert(_ptr(aos), C.byref(layout), C.byref(cells.struct),
                             VIEWS.get(view, view), C.byref(soa.prec), C.byref(soa.struct),
                             _stream(stream)))


def convert_host(aos_np: np.ndarray, layout, cells: DeviceCells, view, soa: DeviceSoa,
                 staging, nthreads=0, stream=None):
    """staging: pinned host uint8 tensor of at least host_staging_size bytes."""
    _check(lib().sph_convert_host(C.c_void_p(aos_np.ctypes.data), C.byref(layout),
                                  C.byref(cells.struct), VIEWS.get(view, view), C.byref(soa.prec),
                                  C.byref(soa.struct), C.c_void_p(staging.data_ptr()),
                                  staging.numel(), int(nthreads), _stream(stream)))


def _np_ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def bin_host(aos_np: np.ndarray, layout, n_c: int, nthreads=0, out=None, hmax=True):
    """Host cell list of the records (sph_bin_host): (cell_start, perm, cell,
    hmax or None) as int32/float32 numpy arrays, or filled into `out`."""
    n = int(aos_np.shape[0])
    Cn = n_c ** 3
    if out is None:
        out = (np.empty(Cn + 1, np.int32), np.empty(n, np.int32), np.empty(n, np.int32),
               np.empty(Cn, np.float32) if hmax else None)
    start, perm, cell, hm = out
    _check(lib().sph_bin_host(C.c_void_p(aos_np.ctypes.data), C.byref(layout), n, int(n_c),
                              _np_ptr(start), _np_ptr(perm), _np_ptr(cell), _np_ptr(hm),
                              int(nthreads)))
    return out


def gather_host(aos_np: np.ndarray, layout, n_c, perm, cell, view, soa: DeviceSoa, staging,
                nthreads=0, stream=None):
    """sph_gather_host: staging is a pinned host uint8 tensor of at least
    host_staging_size bytes; the H2D copies are enqueued on `stream`."""
    _check(lib().sph_gather_host(C.c_void_p(aos_np.ctypes.data), C.byref(layout),
                                 int(aos_np.shape[0]), int(n_c), _np_ptr(perm), _np_ptr(cell),
                                 VIEWS.get(view, view), C.byref(soa.prec), C.byref(soa.struct),
                                 C.c_void_p(staging.data_ptr()), staging.numel(), int(nthreads),
                                 _stream(stream)))


def writeback_host_size(n, view) -> int:
    out = C.c_size_t()
    _check(lib().sph_writeback_host_size(int(n), VIEWS.get(view, view), C.byref(out)))
    return out.value


def writeback_host(soa: DeviceSoa, perm, view, aos_np: np.ndarray, layout, staging, nthreads=0,
                   stream=None):
    """sph_writeback_host (blocking): the view's outputs into the host records."""
    _check(lib().sph_writeback_host(C.byref(soa.struct), int(aos_np.shape[0]), _np_ptr(perm),
                                    VIEWS.get(view, view), C.c_void_p(aos_np.ctypes.data),
                                    C.byref(layout), C.c_void_p(staging.data_ptr()),
                                    staging.numel(), int(nthreads), _stream(stream)))


def writeback(soa: DeviceSoa, cells: DeviceCells, view, aos, layout, stream=None):
    _check(lib().sph_writeback(C.byref(soa.struct), C.byref(cells.struct), VIEWS.get(view, view),
                               _ptr(aos), C.byref(layout), _stream(stream)))


def density(soa: DeviceSoa, cells: DeviceCells, prm=None, til=None, stream=None, work=None):
    _check(lib().sph_density(C.byref(soa.struct), C.byref(soa.prec), C.byref(cells.struct),
                             C.byref(prm or params()), til or Tile(0, 0), _wk(work),
                             _stream(stream)))


def force(soa: DeviceSoa, cells: DeviceCells, prm=None, til=None, stream=None, work=None):
    _check(lib().sph_force(C.byref(soa.struct), C.byref(soa.prec), C.byref(cells.struct),
                           C.byref(prm or params()), til or Tile(0, 0), _wk(work),
                           _stream(stream)))


ETA = 1.2348


def smoothing_length_workspace_size(n: int) -> int:
    out = C.c_size_t()
    _check(lib().sph_smoothing_length_workspace_size(int(n), C.byref(out)))
    return out.value


def smoothing_length(soa, cells, prm=None, eta=ETA, tol=1e-4, max_iter=30, til=None,
                     work=None, ws=None, aos=None, layout=None, stream=None):
    """Iterate every slot's h to the root of h = eta (m / rho(h))^(1/3)
    (sph_smoothing_length); returns (passes, particles not converged)."""
    import torch
    if ws is None:
        ws = torch.empty(smoothing_length_workspace_size(cells.n), dtype=torch.uint8,
                         device=cells.cell_start.device)
    it, left = C.c_int32(), C.c_int32()
    _check(lib().sph_smoothing_length(C.byref(soa.struct), C.byref(soa.prec),
                                      C.byref(cells.struct), C.byref(prm or params()),
                                      float(eta), float(tol), int(max_iter), til or Tile(0, 0),
                                      _wk(work), _ptr(ws), int(ws.numel()), _ptr(aos),
                                      C.byref(layout) if layout is not None else None,
                                      C.byref(it), C.byref(left), _stream(stream)))
    return it.value, left.value


SCHED_NAMES = {-1: None, 0: "grid", 1: "static", 2: "dynamic"}


def tune_candidates():
    """The library's default candidate set: [(ti, k, sched), ...] with sched
    None (one workgroup per cell) or a schedule name."""
    n = C.c_int32()
    _check(lib().sph_tune_candidates(None, 0, C.byref(n)))
    arr = (TuneEntry * n.value)()
    _check(lib().sph_tune_candidates(arr, n.value, C.byref(n)))
    return [(e.tile.ti, e.tile.k, SCHED_NAMES[e.sched]) for e in arr]


def autotune(loop: str, soa: "DeviceSoa", cells: "DeviceCells", prm=None, cand=None, reps=3,
             work_buf=None, stream=None):
    """Time each candidate (ti, k, sched) of the density or force loop
    ('density' / 'force') through sph_autotune; returns ([(ti, k, sched, ms)],
    index of the fastest)."""
    cand = cand if cand is not None else tune_candidates()
    arr = (TuneEntry * len(cand))()
    inv = {v: k for k, v in SCHED_NAMES.items()}
    for e, (ti, k, sc) in zip(arr, cand):
        e.tile = Tile(ti, k)
        e.sched = inv[sc]
        e.ms = -1.0
    best = C.c_int32(-1)
    nbytes = int(work_buf.numel()) if work_buf is not None else 0
    _check(lib().sph_autotune({"density": 0, "force": 1}[loop], C.byref(soa.struct),
                              C.byref(soa.prec), C.byref(cells.struct), C.byref(prm or params()),
                              arr, len(cand), int(reps), _ptr(work_buf), nbytes, C.byref(best),
                              _stream(stream)))
    return [(e.tile.ti, e.tile.k, SCHED_NAMES[e.sched], float(e.ms)) for e in arr], best.value


def kick_drift(soa: DeviceSoa, cells: DeviceCells, dt_kick, dt_drift, moved=None, stream=None):
    _check(lib().sph_kick_drift(C.byref(soa.struct), C.byref(cells.struct), float(dt_kick),
                                float(dt_drift), _ptr(moved), _stream(stream)))


C_CFL = 0.1    # Courant factor of the leapfrog runs' time step


def predict(soa: DeviceSoa, cells: DeviceCells, aos, layout, dt_half, stream=None):
    _check(lib().sph_predict(C.byref(soa.struct), C.byref(soa.prec), C.byref(cells.struct),
                             _ptr(aos), C.byref(layout), float(dt_half), _stream(stream)))


def step_totals(soa: DeviceSoa, cells: DeviceCells, out, workspace, prm=None, c_cfl=C_CFL,
                stream=None):
    """out (8 doubles on the device): sum m v (3), sum m |v|^2/2, sum m u,
    sum m, the Courant step, the number of slots with vsig > 0."""
    _check(lib().sph_step_totals(C.byref(soa.struct), C.byref(soa.prec), C.byref(cells.struct),
                                 C.byref(prm or params()), float(c_cfl), _ptr(out),
                                 _ptr(workspace), workspace.numel() * workspace.element_size(),
                                 _stream(stream)))


def reduce(soa: DeviceSoa, cells: DeviceCells, out, workspace, stream=None):
    _check(lib().sph_reduce(C.byref(soa.struct), C.byref(soa.prec), C.byref(cells.struct),
                            _ptr(out), _ptr(workspace), workspace.numel() * workspace.element_size(),
                            _stream(stream)))


def reduce_aos(aos, layout, cells: DeviceCells, out, workspace, stream=None):
    """sph_reduce_aos: the reductions of reduce() over the AoS records in
    slot order."""
    _check(lib().sph_reduce_aos(_ptr(aos), C.byref(layout), C.byref(cells.struct), _ptr(out),
                                _ptr(workspace), workspace.numel() * workspace.element_size(),
                                _stream(stream)))


def reduce_static(soa: DeviceSoa, cells: DeviceCells, out, stream=None):
    """sph_reduce_static: the reductions of reduce() with the library's own
    device scratch (no workspace, nothing allocated)."""
    _check(lib().sph_reduce_static(C.byref(soa.struct), C.byref(soa.prec), C.byref(cells.struct),
                                   _ptr(out), _stream(stream)))


def density_aos(aos, layout, cells: DeviceCells, prm=None, til=None, stream=None, work=None):
    _check(lib().sph_density_aos(_ptr(aos), C.byref(layout), C.byref(cells.struct),
                                 C.byref(prm or params()), til or Tile(0, 0), _wk(work),
                                 _stream(stream)))


def force_aos(aos, layout, cells: DeviceCells, prm=None, til=None, stream=None, work=None):
    _check(lib().sph_force_aos(_ptr(aos), C.byref(layout), C.byref(cells.struct),
                               C.byref(prm or params()), til or Tile(0, 0), _wk(work),
                               _stream(stream)))


def kick_drift_aos(aos, layout, cells: DeviceCells, dt_kick, dt_drift, moved=None, stream=None):
    _check(lib().sph_kick_drift_aos(_ptr(aos), C.byref(layout), C.byref(cells.struct),
                                    float(dt_kick), float(dt_drift), _ptr(moved), _stream(stream)))


PROBES = {"copy": 0, "read": 1, "write": 2}


def hbm_probe(mode: str, src, dst, nbytes: int, stream=None):
    """sph_hbm_probe: one streaming launch over nbytes ('copy', 'read',
    'write'); src/dst are torch device tensors (or None where unused)."""
    _check(lib().sph_hbm_probe(PROBES[mode], _ptr(src), _ptr(dst), int(nbytes), _stream(stream)))


def sync(stream=None):
    _check(lib().sph_sync(_stream(stream)))
