"""Seeded synthetic particle sets and AoS record packing.

This module holds no SPH arithmetic: it draws particle positions, velocities,
masses, smoothing lengths and internal energies from seeded distributions and
packs them into array-of-structs records. Both the FP64 CPU oracle (tests) and
the HIP path (tests, bench) consume what it produces.

Workloads (paper, Sec. 2 and Sec. 6): a periodic unit box, particles grouped
into spatially co-located buffers of about 64, FP32 fields with FP64 positions
and a 64-bit ID in the AoS record (Table 1 lists the fields).

Recipes:
  * lattice: ``n_side**3`` sites at ``(i + 1/2) * dx`` plus a uniform jitter of
    +-0.1 dx per axis; equal masses ``1/N``; ``u = 1``; velocities
    ``N(0, 0.01**2)`` per component; uniform ``h = eta * dx``.
  * clustered: a uniform background plus 8 periodic Gaussian blobs; ``h``
    follows the analytic number density of the sampling distribution,
    ``h = eta * n(x)**(-1/3)`` (a smooth stand-in for a density iteration).
"""
from __future__ import annotations

import dataclasses

import numpy as np

ETA = 1.2348          # resolution parameter eta (h = eta * mean spacing)

# --------------------------------------------------------------------------
# AoS record layouts (Table 1 plus an int64 ID, FP64 positions)
# --------------------------------------------------------------------------
# FP32 record: 128 bytes, one cache line.
AOS_F32 = np.dtype([
    ("id", "<i8"), ("x", "<f8", (3,)), ("v", "<f4", (3,)), ("a", "<f4", (3,)),
    ("m", "<f4"), ("h", "<f4"), ("u", "<f4"), ("rho", "<f4"), ("P", "<f4"),
    ("c", "<f4"), ("du", "<f4"), ("dt", "<f4"), ("rho_dh", "<f4"),
    ("wcount", "<f4"), ("f", "<f4"), ("vsig", "<f4"), ("div_v", "<f4"),
    ("nngb", "<i4"), ("nforce", "<i4"), ("cell", "<i4"), ("pad", "V8"),
], align=False)
assert AOS_F32.itemsize == 128

# FP64 record: every floating field in double precision, 200 bytes.
AOS_F64 = np.dtype([
    ("id", "<i8"), ("x", "<f8", (3,)), ("v", "<f8", (3,)), ("a", "<f8", (3,)),
    ("m", "<f8"), ("h", "<f8"), ("u", "<f8"), ("rho", "<f8"), ("P", "<f8"),
    ("c", "<f8"), ("du", "<f8"), ("dt", "<f8"), ("rho_dh", "<f8"),
    ("wcount", "<f8"), ("f", "<f8"), ("vsig", "<f8"), ("div_v", "<f8"),
    ("nngb", "<i4"), ("nforce", "<i4"), ("cell", "<i4"), ("pad", "V4"),
], align=False)
assert AOS_F64.itemsize == 200


@dataclasses.dataclass
class ParticleSet:
    """Plain FP64 particle fields in input order."""
    x: np.ndarray      # (N, 3) positions in [0, 1)
    v: np.ndarray      # (N, 3) velocities
    m: np.ndarray      # (N,)   masses
    h: np.ndarray      # (N,)   smoothing lengths
    u: np.ndarray      # (N,)   specific internal energies
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def subset(self, idx) -> "ParticleSet":
        idx = np.asarray(idx)
        return ParticleSet(self.x[idx].copy(), self.v[idx].copy(), self.m[idx].copy(),
                           self.h[idx].copy(), self.u[idx].copy(), self.name)

    def rounded_to(self, kind: str) -> "ParticleSet":
        """The values an AoS record of ``kind`` ('f32' or 'f64') holds, as FP64.
        Positions stay FP64 in both records."""
        if kind == "f64":
            return self
        r = lambda a: a.astype(np.float32).astype(np.float64)
        return ParticleSet(self.x.copy(), r(self.v), r(self.m), r(self.h), r(self.u), self.name)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def lattice_set(n_side: int, seed: int, *, jitter: float = 0.1, v_sigma: float = 0.01,
                u0: float = 1.0, eta: float = ETA, order: str = "blocked", block: int = 4,
                perfect: bool = False) -> ParticleSet:
    """Jittered cubic lattice of ``n_side**3`` particles in the periodic unit box.

    order: 'raster' (x fastest), 'blocked' (sites enumerated block by block of
    ``block**3`` lattice sites, i.e. contiguous buffers of spatially co-located
    particles), or 'shuffled' (a seeded random permutation).
    perfect: no jitter and zero velocities (closed-form lattice cases).
    """
    rng = _rng(seed)
    n = n_side ** 3
    dx = 1.0 / n_side
    k = np.arange(n_side)
    gz, gy, gx = np.meshgrid(k, k, k, indexing="ij")            # x fastest
    site = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    x = (site.astype(np.float64) + 0.5) * dx
    if perfect:
        v = np.zeros((n, 3))
    else:
        x = x + rng.uniform(-jitter, jitter, size=(n, 3)) * dx
        v = rng.normal(0.0, v_sigma, size=(n, 3))
    x = np.mod(x, 1.0)
    m = np.full(n, 1.0 / n)
    h = np.full(n, eta * dx)
    u = np.full(n, float(u0))
    if order == "raster":
        perm = np.arange(n)
    elif order == "blocked":
        if n_side % block:
            raise ValueError("n_side must be a multiple of block")
        nb = n_side // block
        b = site // block
        w = site % block
        key = ((b[:, 2] * nb + b[:, 1]) * nb + b[:, 0]) * block ** 3 + \
              (w[:, 2] * block + w[:, 1]) * block + w[:, 0]
        perm = np.argsort(key, kind="stable")
    elif order == "shuffled":
        perm = rng.permutation(n)
    else:
        raise ValueError(order)
    return ParticleSet(x[perm], v[perm], m[perm], h[perm], u[perm],
                       name=f"lattice{n_side}_s{seed}")


def blob_centres(seed: int, nblobs: int = 8) -> np.ndarray:
    return _rng(seed * 7919 + 17).uniform(0.0, 1.0, size=(nblobs, 3))


def clustered_number_density(x: np.ndarray, n_total: int, f_blob: float, centres: np.ndarray,
                             sigma: float) -> np.ndarray:
    """Analytic number density of the clustered sampling distribution (periodic
    Gaussian blobs, images within +-1 box, over a uniform background)."""
    nb = centres.shape[0]
    dens = np.full(x.shape[0], n_total * (1.0 - f_blob))
    norm = n_total * f_blob / nb / ((2.0 * np.pi) ** 1.5 * sigma ** 3)
    for c in centres:
        d = x - c
        d -= np.rint(d)
        dens += norm * np.exp(-0.5 * np.einsum("ij,ij->i", d, d) / sigma ** 2)
    return dens


def clustered_set(n: int, seed: int, *, f_blob: float = 0.22, sigma: float = 0.03,
                  nblobs: int = 8, v_sigma: float = 0.01, u0: float = 1.0,
                  eta: float = ETA) -> ParticleSet:
    """Uniform background plus ``nblobs`` periodic Gaussian blobs.

    Masses are equal (``1/n`` rounded to a power of two when ``n`` is one);
    ``h`` follows the analytic number density of the sampling distribution.
    Particles are ordered by a coarse 16**3 block key, so the AoS holds
    spatially grouped buffers as in the paper's setup.
    """
    rng = _rng(seed)
    centres = blob_centres(seed, nblobs)
    nblob = int(round(f_blob * n))
    nb_each = np.full(nblobs, nblob // nblobs)
    nb_each[: nblob % nblobs] += 1
    parts = [rng.uniform(0.0, 1.0, size=(n - nblob, 3))]
    for c, k in zip(centres, nb_each):
        parts.append(c + rng.normal(0.0, sigma, size=(k, 3)))
    x = np.mod(np.concatenate(parts, axis=0), 1.0)
    v = rng.normal(0.0, v_sigma, size=(n, 3))
    m = np.full(n, 1.0 / n)
    nd = clustered_number_density(x, n, f_blob, centres, sigma)
    h = eta * nd ** (-1.0 / 3.0)
    u = np.full(n, float(u0))
    g = np.minimum((x * 16).astype(np.int64), 15)
    key = (g[:, 2] * 16 + g[:, 1]) * 16 + g[:, 0]
    perm = np.argsort(key, kind="stable")
    return ParticleSet(x[perm], v[perm], m[perm], h[perm], u[perm],
                       name=f"clustered{n}_s{seed}")


def pack_aos(ps: ParticleSet, kind: str = "f32") -> np.ndarray:
    """Pack a particle set into AoS records ('f32': 128-byte record with FP32
    fields and FP64 positions; 'f64': 200-byte all-FP64 record)."""
    dt = AOS_F32 if kind == "f32" else AOS_F64
    rec = np.zeros(ps.n, dtype=dt)
    rec["id"] = np.arange(ps.n, dtype=np.int64)
    rec["x"] = ps.x
    rec["v"] = ps.v
    rec["m"] = ps.m
    rec["h"] = ps.h
    rec["u"] = ps.u
    rec["cell"] = -1
    return rec


def unpack_aos(rec: np.ndarray) -> ParticleSet:
    f = lambda a: np.asarray(a, dtype=np.float64)
    return ParticleSet(f(rec["x"]).copy(), f(rec["v"]).copy(), f(rec["m"]).copy(),
                       f(rec["h"]).copy(), f(rec["u"]).copy())


# Named workloads: the small lattice, the 128**3 lattice and the clustered set.
def small_set(seed: int = 1, order: str = "shuffled") -> ParticleSet:
    """4,096 particles on a jittered 16**3 lattice."""
    return lattice_set(16, seed, order=order)


def medium_set(seed: int = 2, order: str = "blocked") -> ParticleSet:
    """2,097,152 particles on a jittered 128**3 lattice."""
    return lattice_set(128, seed, order=order)


def clustered_k_set(seed: int = 3) -> ParticleSet:
    """4,194,304 particles, 19 % of them in 8 periodic Gaussian blobs
    (sigma 0.03) over a uniform background. With h from the density
    iteration and cells as small as the largest support radius allows
    (48 per axis) the occupancy spans about 10 to 2,000 particles per cell
    (median 30); the blob fraction is chosen for that upper end."""
    return clustered_set(1 << 22, seed, f_blob=0.19)
