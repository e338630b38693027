"""Python front end of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark. The product path never imports it.

Functions take and return plain numpy arrays in input (generator) order.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

F32, F16, BF16, F64 = 0, 1, 2, 3
DTYPE_CODES = {"f32": F32, "f16": F16, "bf16": BF16, "f64": F64}
TRUNC = 0x100
# truncate_mantissa storage of T bits in total: "t9" ... "t64"
DTYPE_CODES.update({f"t{T}": TRUNC + T for T in range(9, 65)})

# Constants of the method (paper Sec. 2.1 names the cubic spline; the values
# are the readings listed in the design notes).
GAMMA_K = 1.825742      # H / h for the 3D cubic spline
GAMMA = 5.0 / 3.0       # ideal-gas adiabatic index
ALPHA = 0.8             # artificial-viscosity strength
BETA = 3.0              # signal-velocity coefficient
ETA = 1.2348            # h = ETA (m / rho)^(1/3): about 48 neighbours
C_CFL = 0.1             # time step = C_CFL * H / v_sig (Courant factor)


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no fast-math, no FP contraction)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    src = os.path.join(HERE, "oracle.c")
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
           "-D_DEFAULT_SOURCE", "-Wall", "-fPIC", "-shared", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Params(C.Structure):
    _fields_ = [("gamma_k", C.c_double), ("gamma", C.c_double), ("alpha", C.c_double),
                ("beta", C.c_double), ("gradh", C.c_int32), ("kernel", C.c_int32)]


KERNEL_M4, KERNEL_WENDLAND_C2 = 0, 1
KERNELS = {"m4": KERNEL_M4, "wendland_c2": KERNEL_WENDLAND_C2}
# support radius over smoothing length of the Wendland C2 function: the
# kernel's standard deviation matches the M4 spline's at equal h
GAMMA_K_WENDLAND_C2 = 1.936492


def params(gamma_k=None, gamma=GAMMA, alpha=ALPHA, beta=BETA, gradh=True, kernel="m4") -> Params:
    k = KERNELS.get(kernel, kernel)
    if gamma_k is None:
        gamma_k = GAMMA_K_WENDLAND_C2 if k == KERNEL_WENDLAND_C2 else GAMMA_K
    return Params(gamma_k, gamma, alpha, beta, 1 if gradh else 0, k)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        d, i32, i64, u16, f32 = (C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                 C.c_int64, C.POINTER(C.c_uint16), C.POINTER(C.c_float))
        L.orc_w_hat.restype = C.c_double
        L.orc_w_hat.argtypes = [C.c_double]
        L.orc_dw_hat.restype = C.c_double
        L.orc_dw_hat.argtypes = [C.c_double]
        L.orc_W.restype = C.c_double
        L.orc_W.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_dWdh.restype = C.c_double
        L.orc_dWdh.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_kernel_w.restype = C.c_double
        L.orc_kernel_w.argtypes = [C.c_int, C.c_double]
        L.orc_kernel_dw.restype = C.c_double
        L.orc_kernel_dw.argtypes = [C.c_int, C.c_double]
        L.orc_bin.argtypes = [C.c_int, d, C.c_int, i32, i32, i32, d]
        u8 = C.POINTER(C.c_uint8)
        L.orc_density.argtypes = [C.c_int, d, d, d, d, C.POINTER(Params), C.c_int, C.c_int,
                                  i32, C.c_int, u8, d, d, d, d, d, d, i32]
        L.orc_force.argtypes = [C.c_int, d, d, d, d, d, d, d, d, C.POINTER(Params), C.c_int,
                                C.c_int, i32, C.c_int, u8, d, d, d, i32]
        L.orc_kick_drift.argtypes = [C.c_int, d, d, d, d, d, C.c_double, C.c_double]
        L.orc_kick_drift.restype = None
        L.orc_reduce.argtypes = [C.c_int, d, d, d, d, d]
        L.orc_reduce.restype = None
        L.orc_near_support.argtypes = [C.c_int, d, d, C.c_double, C.c_int, C.c_int, i32, C.c_int,
                                       C.c_double, C.c_double, i32, i32]
        L.orc_pos_offsets.argtypes = [C.c_int, d, C.c_int, C.c_int, d, C.POINTER(C.c_uint8)]
        L.orc_f32_to_f16.restype = C.c_uint16
        L.orc_f32_to_f16.argtypes = [C.c_float]
        L.orc_f16_to_f32.restype = C.c_float
        L.orc_f16_to_f32.argtypes = [C.c_uint16]
        L.orc_f32_to_bf16.restype = C.c_uint16
        L.orc_f32_to_bf16.argtypes = [C.c_float]
        L.orc_bf16_to_f32.restype = C.c_float
        L.orc_bf16_to_f32.argtypes = [C.c_uint16]
        L.orc_quant_array.argtypes = [i64, f32, u16, C.c_int]
        L.orc_quant_array.restype = None
        L.orc_dequant_array.argtypes = [i64, u16, f32, C.c_int]
        L.orc_dequant_array.restype = None
        L.orc_roundtrip.restype = C.c_double
        L.orc_roundtrip.argtypes = [C.c_double, C.c_int, C.c_int]
        L.orc_dequantise_set.argtypes = [C.c_int, d, d, d, d, d, C.c_int, C.c_int, C.c_int,
                                         C.c_int, i32, C.c_int, d, d, d, d, d]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_bin_sub.argtypes = [C.c_int, d, C.c_int, C.c_int, i32, i32, i32]
        L.orc_smoothing_length.argtypes = [C.c_int, d, d, d, C.c_double, C.POINTER(Params),
                                           C.c_int, C.c_int, C.c_double, C.c_double, C.c_int,
                                           i32, C.c_int, d, i32]
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the following OpenMP regions (timing runs)."""
    lib().orc_set_threads(int(n))


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def w_hat(u: float, kernel="m4") -> float:
    return lib().orc_kernel_w(KERNELS.get(kernel, kernel), float(u))


def dw_hat(u: float, kernel="m4") -> float:
    return lib().orc_kernel_dw(KERNELS.get(kernel, kernel), float(u))


def W(r, h, gamma_k=GAMMA_K):
    return lib().orc_W(float(r), float(h), float(gamma_k))


def dWdh(r, h, gamma_k=GAMMA_K):
    return lib().orc_dWdh(float(r), float(h), float(gamma_k))


def bin_cells(x, n_c):
    """-> (cell[N], cell_start[C+1], perm[N], off[N,3])"""
    x = _f64(x)
    n = x.shape[0]
    cell = np.empty(n, np.int32)
    start = np.empty(n_c ** 3 + 1, np.int32)
    perm = np.empty(n, np.int32)
    off = np.empty((n, 3), np.float64)
    rc = lib().orc_bin(n, _p(x, C.c_double), n_c, _p(cell, C.c_int32), _p(start, C.c_int32),
                       _p(perm, C.c_int32), _p(off, C.c_double))
    assert rc == 0
    return cell, start, perm, off


def bin_sub(x, n_c, sub_bits):
    """-> (key[N], sub_start[n_c^3 R^3 + 1], perm[N]) with R = 2**sub_bits"""
    x = _f64(x)
    n = x.shape[0]
    R = 1 << sub_bits
    key = np.empty(n, np.int32)
    start = np.empty(n_c ** 3 * R ** 3 + 1, np.int32)
    perm = np.empty(n, np.int32)
    rc = lib().orc_bin_sub(n, _p(x, C.c_double), n_c, sub_bits, _p(key, C.c_int32),
                           _p(start, C.c_int32), _p(perm, C.c_int32))
    assert rc == 0
    return key, start, perm


def _mask(jmask):
    return None if jmask is None else np.ascontiguousarray(jmask, dtype=np.uint8)


def density(ps, prm=None, mode="cells", n_c=None, sel=None, jmask=None):
    """FP64 density loop. Returns a dict of arrays (length N, or len(sel)).
    jmask (bool per particle) restricts the neighbours j to a subset: the
    sums over one cell pair, as a serving task computes them."""
    prm = prm or params()
    x, m, h, u = _f64(ps.x), _f64(ps.m), _f64(ps.h), _f64(ps.u)
    n = x.shape[0]
    if sel is not None:
        sel = np.ascontiguousarray(sel, dtype=np.int32)
    cnt = n if sel is None else sel.shape[0]
    out = {k: np.empty(cnt) for k in ("rho", "wcount", "rho_dh", "f", "P", "c")}
    out["nngb"] = np.empty(cnt, np.int32)
    md = 0 if mode == "brute" else 1
    rc = lib().orc_density(n, _p(x, C.c_double), _p(m, C.c_double), _p(h, C.c_double),
                           _p(u, C.c_double), C.byref(prm), md, int(n_c or 0),
                           _p(sel, C.c_int32), cnt, _p(_mask(jmask), C.c_uint8),
                           *[_p(out[k], C.c_double) for k in ("rho", "wcount", "rho_dh", "f",
                                                               "P", "c")],
                           _p(out["nngb"], C.c_int32))
    if rc != 0:
        raise ValueError(f"orc_density failed ({rc}): cell side must be >= max H and n_c >= 3")
    return out


def force(ps, dens, prm=None, mode="cells", n_c=None, sel=None, jmask=None):
    """FP64 force loop; ``dens`` holds rho, f, P, c over all particles.
    jmask as for density()."""
    prm = prm or params()
    x, v, m, h = _f64(ps.x), _f64(ps.v), _f64(ps.m), _f64(ps.h)
    n = x.shape[0]
    if sel is not None:
        sel = np.ascontiguousarray(sel, dtype=np.int32)
    cnt = n if sel is None else sel.shape[0]
    a = np.empty((cnt, 3))
    du = np.empty(cnt)
    vsig = np.empty(cnt)
    nf = np.empty(cnt, np.int32)
    arr = [_f64(dens[k]) for k in ("rho", "f", "P", "c")]
    md = 0 if mode == "brute" else 1
    rc = lib().orc_force(n, _p(x, C.c_double), _p(v, C.c_double), _p(m, C.c_double),
                         _p(h, C.c_double), *[_p(t, C.c_double) for t in arr], C.byref(prm),
                         md, int(n_c or 0), _p(sel, C.c_int32), cnt, _p(_mask(jmask), C.c_uint8),
                         _p(a, C.c_double),
                         _p(du, C.c_double), _p(vsig, C.c_double), _p(nf, C.c_int32))
    if rc != 0:
        raise ValueError(f"orc_force failed ({rc})")
    return {"a": a, "du": du, "vsig": vsig, "nforce": nf}


def kick_drift(x, v, u, a, du, dt_kick, dt_drift):
    x, v, u = _f64(x).copy(), _f64(v).copy(), _f64(u).copy()
    a, du = _f64(a), _f64(du)
    lib().orc_kick_drift(x.shape[0], _p(x, C.c_double), _p(v, C.c_double), _p(u, C.c_double),
                         _p(a, C.c_double), _p(du, C.c_double), float(dt_kick), float(dt_drift))
    return x, v, u


def reduce(m, v, a, du):
    out = np.empty(6)
    m, v, a, du = _f64(m), _f64(v), _f64(a), _f64(du)
    lib().orc_reduce(m.shape[0], _p(m, C.c_double), _p(v, C.c_double), _p(a, C.c_double),
                     _p(du, C.c_double), _p(out, C.c_double))
    return out


# Pairs this close to a support radius may be decided either way by a count
# taken in FP32 on stored offsets (the kernels' rounding of the shifted
# positions and of r^2 and H^2 stays well inside both terms).
NEAR_EPS_REL = 1e-5
NEAR_EPS_ABS_CELLS = 2.0 ** -18     # times the cell side


def near_support(ps, n_c, gamma_k=GAMMA_K, mode="cells", sel=None, eps_rel=NEAR_EPS_REL,
                 eps_abs=None):
    """Per particle (or per entry of sel): the number of density-list pairs
    with |r - H_i| < eps_rel H_i + eps_abs and of force-list pairs within
    that distance of H_i or H_j (eps_abs: NEAR_EPS_ABS_CELLS / n_c by
    default) -> (near_density, near_force)."""
    x, h = _f64(ps.x), _f64(ps.h)
    n = x.shape[0]
    if eps_abs is None:
        eps_abs = NEAR_EPS_ABS_CELLS / n_c
    if sel is not None:
        sel = np.ascontiguousarray(sel, dtype=np.int32)
    cnt = n if sel is None else sel.shape[0]
    nd = np.empty(cnt, np.int32)
    nf = np.empty(cnt, np.int32)
    rc = lib().orc_near_support(n, _p(x, C.c_double), _p(h, C.c_double), float(gamma_k),
                                0 if mode == "brute" else 1, int(n_c), _p(sel, C.c_int32), cnt,
                                float(eps_rel), float(eps_abs), _p(nd, C.c_int32),
                                _p(nf, C.c_int32))
    if rc != 0:
        raise ValueError(f"orc_near_support failed ({rc})")
    return nd, nf


def pos_offsets(x, n_c, anchor=0):
    """(off[N, 3], code[N]): FP64 offsets of the wrapped positions from their
    anchor (0: cell corner; 1 + b: centre of the sub-cell of side
    1/(n_c 2^b)) and the anchor sub-cell code a_x + 4 a_y + 16 a_z."""
    x = _f64(x)
    n = x.shape[0]
    off = np.empty((n, 3))
    code = np.empty(n, np.uint8)
    rc = lib().orc_pos_offsets(n, _p(x, C.c_double), int(n_c), int(anchor), _p(off, C.c_double),
                               _p(code, C.c_uint8))
    assert rc == 0
    return off, code


def quant(a32, dtype):
    a32 = np.ascontiguousarray(a32, dtype=np.float32)
    out = np.empty(a32.shape, np.uint16)
    lib().orc_quant_array(a32.size, _p(a32, C.c_float), _p(out, C.c_uint16), DTYPE_CODES[dtype])
    return out


def dequant(bits, dtype):
    bits = np.ascontiguousarray(bits, dtype=np.uint16)
    out = np.empty(bits.shape, np.float32)
    lib().orc_dequant_array(bits.size, _p(bits, C.c_uint16), _p(out, C.c_float),
                            DTYPE_CODES[dtype])
    return out


def roundtrip(v, dtype, scale=0):
    return lib().orc_roundtrip(float(v), DTYPE_CODES[dtype], int(scale))


def dequantise_set(ps, n_c, pos="f32", vel="f32", mhu="f32", scales=(0, 0, 0), anchor=0):
    """The particle set as an SoA view of the given storage formats holds it,
    read back into FP64 (positions = anchor + stored offset; anchor as in
    pos_offsets)."""
    from paper_2512_05516_amd.inputs import ParticleSet
    x, v, m, h, u = (_f64(ps.x), _f64(ps.v), _f64(ps.m), _f64(ps.h), _f64(ps.u))
    n = x.shape[0]
    xq, vq = np.empty_like(x), np.empty_like(v)
    mq, hq, uq = np.empty_like(m), np.empty_like(h), np.empty_like(u)
    sc = np.ascontiguousarray(scales, dtype=np.int32)
    rc = lib().orc_dequantise_set(n, _p(x, C.c_double), _p(v, C.c_double), _p(m, C.c_double),
                                  _p(h, C.c_double), _p(u, C.c_double), int(n_c),
                                  DTYPE_CODES[pos], DTYPE_CODES[vel], DTYPE_CODES[mhu],
                                  _p(sc, C.c_int32), int(anchor), _p(xq, C.c_double),
                                  _p(vq, C.c_double), _p(mq, C.c_double), _p(hq, C.c_double),
                                  _p(uq, C.c_double))
    assert rc == 0
    return ParticleSet(xq, vq, mq, hq, uq, ps.name + "_dq")


def smoothing_length(ps, eta=ETA, h_max=None, tol=1e-4, max_iter=30, prm=None, mode="cells",
                     n_c=None, sel=None):
    """Per-particle roots of h = eta (m / rho(h))^(1/3) by limited Newton
    steps from ps.h. Returns (h, iterations); iterations = max_iter + 1
    marks a particle that did not converge."""
    prm = prm or params()
    x, m, h0 = _f64(ps.x), _f64(ps.m), _f64(ps.h)
    n = x.shape[0]
    if h_max is None:
        h_max = 1.0 / (prm.gamma_k * n_c) if n_c else np.inf
    if sel is not None:
        sel = np.ascontiguousarray(sel, dtype=np.int32)
    cnt = n if sel is None else sel.shape[0]
    h = np.empty(cnt)
    it = np.empty(cnt, np.int32)
    rc = lib().orc_smoothing_length(n, _p(x, C.c_double), _p(m, C.c_double), _p(h0, C.c_double),
                                    float(eta), C.byref(prm), 0 if mode == "brute" else 1,
                                    int(n_c or 0), float(h_max), float(tol), int(max_iter),
                                    _p(sel, C.c_int32), cnt, _p(h, C.c_double),
                                    _p(it, C.c_int32))
    if rc != 0:
        raise ValueError(f"orc_smoothing_length failed ({rc}): gamma_k h_max must fit a cell")
    return h, it


def task_partials(ps, n_c, tasks, dens, prm=None, perm=None, cell=None):
    """Partial sums of serving tasks (one cell pair each): for task
    (kind, ci, cj, i_begin, i_end) the density (kind 0) or force (kind 1)
    sums over i = perm[i_begin:i_end] (sorted-slot order of the cell list)
    and j restricted to cell cj, evaluated by density()/force() with that j
    subset. dens: full density outputs (rho, f, P, c) over all particles.
    Returns a list of dicts, one per task."""
    if perm is None or cell is None:
        cell, _, perm, _ = bin_cells(ps.x, n_c)
    out = []
    for (kind, ci, cj, ib, ie) in tasks:
        sel = perm[ib:ie]
        jm = cell == cj
        if kind == 0:
            d = density(ps, prm, n_c=n_c, sel=sel, jmask=jm)
            out.append({"rho": d["rho"], "wcount": d["wcount"], "rho_dh": d["rho_dh"],
                        "count": d["nngb"]})
        else:
            f = force(ps, dens, prm, n_c=n_c, sel=sel, jmask=jm)
            out.append({"a": f["a"], "du": f["du"], "vsig": f["vsig"], "count": f["nforce"]})
    return out


# ---------------------------------------------------------------------------
# Time integration: CFL time step, conserved totals and the leapfrog
# kick-drift-kick over several steps (the paper's Kick and Drift kernels,
# Sec. 6, arranged as the second-order symplectic integrator). Plain FP64
# compositions of the loops above.
# ---------------------------------------------------------------------------

def timestep(h, vsig, c_cfl=C_CFL, gamma_k=GAMMA_K):
    """Per-particle Courant time step c_cfl * (gamma_k h) / vsig (inf where
    vsig = 0: a particle without neighbours sets no limit) and the global
    minimum, the single step size of the whole run."""
    h, vsig = _f64(h), _f64(vsig)
    dt = np.full(h.shape, np.inf)
    ok = vsig > 0.0
    dt[ok] = c_cfl * (gamma_k * h[ok]) / vsig[ok]
    return dt, (float(dt.min()) if dt.size else np.inf)


def totals(m, v, u):
    """Momentum sum m v (3), kinetic sum m |v|^2 / 2, thermal sum m u, mass."""
    m, v, u = _f64(m), _f64(v), _f64(u)
    return {"p": (m[:, None] * v).sum(0), "ekin": float(0.5 * (m * (v * v).sum(1)).sum()),
            "eth": float((m * u).sum()), "mass": float(m.sum())}


def kdk_run(ps, n_c, steps, dt=None, c_cfl=C_CFL, prm=None, mode="cells"):
    """Leapfrog kick-drift-kick with h held fixed. Forces at the start;
    each step takes the step size (dt, or the CFL minimum from the last
    forces), kicks v and u by half a step with the last rates, drifts x by
    a whole step with the kicked v, evaluates density and force at the new
    positions with v and u predicted to the end of the step by the last
    rates (v + a dt/2, u + du dt/2: the forces depend on v through the
    viscosity and on u through the pressure), and kicks the half-step v and
    u by the second half with the new rates. Returns (final ParticleSet,
    history): history[k] holds the step size and the totals before step k,
    the last entry the totals after the run (dt None)."""
    from paper_2512_05516_amd.inputs import ParticleSet
    prm = prm or params()
    x, v, u = _f64(ps.x).copy(), _f64(ps.v).copy(), _f64(ps.u).copy()
    m, h = _f64(ps.m), _f64(ps.h)
    at = lambda vv, uu: ParticleSet(x, vv, m, h, uu, ps.name)
    d = density(at(v, u), prm, mode=mode, n_c=n_c)
    f = force(at(v, u), d, prm, mode=mode, n_c=n_c)
    hist = []
    for _ in range(steps):
        step = dt if dt is not None else timestep(h, f["vsig"], c_cfl, prm.gamma_k)[1]
        hist.append(dict(totals(m, v, u), dt=step))
        a0, du0 = f["a"], f["du"]
        x, v, u = kick_drift(x, v, u, a0, du0, 0.5 * step, step)
        vp, up = v + a0 * (0.5 * step), u + du0 * (0.5 * step)
        d = density(at(vp, up), prm, mode=mode, n_c=n_c)
        f = force(at(vp, up), d, prm, mode=mode, n_c=n_c)
        x, v, u = kick_drift(x, v, u, f["a"], f["du"], 0.5 * step, 0.0)
    hist.append(dict(totals(m, v, u), dt=None))
    return at(v, u), hist
