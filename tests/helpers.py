"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI,
evaluate the oracle on the same inputs, and the error norms (relative RMSE
normalised by the mean magnitude, as in the paper's Sec. 7)."""
import numpy as np


def rel_rmse(got, ref):
    """sqrt(mean |got - ref|^2) / mean |ref| (vectors: Euclidean norms)."""
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    if ref.ndim == 2:
        d = np.linalg.norm(got - ref, axis=1)
        r = np.linalg.norm(ref, axis=1)
    else:
        d, r = np.abs(got - ref), np.abs(ref)
    return float(np.sqrt((d ** 2).mean()) / r.mean())


def rel_max(got, ref):
    """max |got - ref| / mean |ref|."""
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    if ref.ndim == 2:
        d = np.linalg.norm(got - ref, axis=1)
        r = np.linalg.norm(ref, axis=1)
    else:
        d, r = np.abs(got - ref), np.abs(ref)
    return float(d.max() / r.mean())


def max_rel(got, ref):
    """max_i |got_i / ref_i - 1|."""
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    return float(np.max(np.abs(got / ref - 1.0)))


def oracle_step(orc, ps, n_c, prm=None, sel=None):
    d = orc.density(ps, prm, n_c=n_c)
    f = orc.force(ps, d, prm, n_c=n_c, sel=sel)
    return d, f


def run_gpu(ps, n_c, kind="f32", prec=None, til=None, prm=None, kick=None, **kw):
    """Pack ps into AoS records of `kind`, run bin, convert(full), density,
    force (and optionally kick/drift + writeback) through the C ABI. kw go to
    Pipeline (sub_bits, sched, til_force)."""
    from paper_2512_05516_amd import inputs, sphmi
    from paper_2512_05516_amd.pipeline import Pipeline
    rec = inputs.pack_aos(ps, kind)
    pipe = Pipeline(rec, n_c, prec=prec, til=til, prm=prm, **kw)
    pipe.bin()
    pipe.convert("full")
    pipe.density()
    pipe.force()
    pipe.reduce()
    if kick is not None:
        pipe.kick_drift(*kick)
    pipe.writeback("full")
    return pipe


def gpu_fields(pipe):
    """Outputs in input (generator) order from the written-back records."""
    r = pipe.records()
    return {k: np.asarray(r[k], np.float64) if r[k].dtype.kind == "f" else r[k].copy()
            for k in ("rho", "wcount", "rho_dh", "f", "P", "c", "nngb", "a", "du", "vsig",
                      "nforce", "x", "v", "u", "cell")}


def brick_order(n_c, b=4):
    """Cell ids in the order the pair launches visit them, enumerated
    directly: bricks of b x b x b cells (thinner at the upper box edge) with
    x the fastest brick index, then y, then z; inside a brick x fastest."""
    out = []
    for z0 in range(0, n_c, b):
        for y0 in range(0, n_c, b):
            for x0 in range(0, n_c, b):
                for z in range(z0, min(z0 + b, n_c)):
                    for y in range(y0, min(y0 + b, n_c)):
                        for x in range(x0, min(x0 + b, n_c)):
                            out.append(x + n_c * (y + n_c * z))
    return np.array(out, dtype=np.int64)


def assert_counts(orc, got_nd, got_nf, ref_nd, ref_nf, ps, n_c, sel=None, gamma_k=None,
                  min_clear=0.9, tag=""):
    """Neighbour counts of the GPU against the FP64 brute-force definition
    (the oracle's nngb / nforce on the set `ps` as the kernels read it):
    equal for every particle with no pair near a support radius (the
    oracle's near_support band, wider than the FP32 rounding of the
    shifted offsets, of r^2 and of H^2); for the others the difference is at
    most the number of such pairs; at least `min_clear` of the particles
    are clear. got_* and ref_* are per entry of sel (all particles if None).
    Returns the fraction of clear particles (density, force)."""
    kw = {} if gamma_k is None else {"gamma_k": gamma_k}
    near_d, near_f = orc.near_support(ps, n_c, sel=sel, **kw)
    got_nd, got_nf = np.asarray(got_nd), np.asarray(got_nf)
    ref_nd, ref_nf = np.asarray(ref_nd), np.asarray(ref_nf)
    cd, cf = near_d == 0, near_f == 0
    assert np.array_equal(got_nd[cd], ref_nd[cd]), (tag, "nngb", np.nonzero(got_nd[cd] != ref_nd[cd]))
    assert np.array_equal(got_nf[cf], ref_nf[cf]), (tag, "nforce", np.nonzero(got_nf[cf] != ref_nf[cf]))
    assert np.all(np.abs(got_nd.astype(np.int64) - ref_nd) <= near_d), tag
    assert np.all(np.abs(got_nf.astype(np.int64) - ref_nf) <= near_f), tag
    fr = (float(cd.mean()) if cd.size else 1.0, float(cf.mean()) if cf.size else 1.0)
    assert fr[0] >= min_clear and fr[1] >= min_clear, (tag, fr)
    return fr


def unpack_trunc(words, T: int, n: int) -> np.ndarray:
    """Reading of n truncated codes of T bits from a packed field (value k at
    bits [kT, kT + T) of little-endian 32-bit words, the layout the header
    defines for SPH_TRUNC_BITS storage), widened to FP32: the code shifted
    back into the top of an IEEE single (T > 16) or half (T <= 16)."""
    w = np.asarray(words).view(np.uint32).astype(np.uint64)
    b = np.arange(n, dtype=np.uint64) * np.uint64(T)
    i = (b >> np.uint64(5)).astype(np.int64)
    v = w[i] | (w[i + 1] << np.uint64(32))
    code = (v >> (b & np.uint64(31))) & np.uint64((1 << T) - 1)
    if T > 16:
        return (code << np.uint64(32 - T)).astype(np.uint32).view(np.float32)
    return (code << np.uint64(16 - T)).astype(np.uint16).view(np.float16).astype(np.float32)
