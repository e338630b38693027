"""Pins of the FP64 oracle against facts fixed outside the oracle itself:
closed forms, conservation laws, a variational identity, brute force, library
routines and the paper's Table 2. Each test names what it pins and which
plausible mistake it would catch."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from paper_2512_05516_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Kernel (Sec. 2.1: cubic spline with compact support)
# --------------------------------------------------------------------------

def test_kernel_normalised(orc):
    # The 3D kernel integrates to one over its unit support: catches a wrong
    # prefactor (e.g. the 1D/2D normalisation) or a wrong polynomial term.
    val, err = integrate.quad(lambda u: 4.0 * math.pi * u * u * orc.w_hat(u), 0.0, 1.0,
                              points=[0.5], epsabs=1e-14, epsrel=1e-14)
    assert abs(val - 1.0) < 1e-12


def test_kernel_continuity_and_support(orc):
    eps = 1e-12
    assert abs(orc.w_hat(0.5 - eps) - orc.w_hat(0.5 + eps)) < 1e-9
    assert abs(orc.dw_hat(0.5 - eps) - orc.dw_hat(0.5 + eps)) < 1e-9
    assert abs(orc.w_hat(0.5) - 2.0 / math.pi) < 1e-15
    assert abs(orc.dw_hat(0.5) + 12.0 / math.pi) < 1e-14
    assert orc.w_hat(1.0) == 0.0 and orc.dw_hat(1.0) == 0.0
    assert orc.w_hat(1.3) == 0.0 and orc.dw_hat(1.3) == 0.0
    assert orc.dw_hat(0.0) == 0.0          # smooth at the origin


def test_kernel_derivative_matches_finite_difference(orc):
    # w_hat' against a central difference of w_hat: catches a sign or
    # coefficient error in the derivative the force loop uses.
    for u in np.linspace(0.01, 0.99, 97):
        if abs(u - 0.5) < 1e-3:
            continue
        d = 1e-6
        fd = (orc.w_hat(u + d) - orc.w_hat(u - d)) / (2 * d)
        assert abs(fd - orc.dw_hat(u)) < 1e-7 * max(1.0, abs(fd))


def test_dWdh_matches_finite_difference(orc):
    # dW/dh at fixed r against a central difference in h.
    for r in np.linspace(0.0, 0.14, 29):
        h = 0.077175
        d = 1e-7 * h
        fd = (orc.W(r, h + d) - orc.W(r, h - d)) / (2 * d)
        got = orc.dWdh(r, h)
        assert abs(fd - got) <= 1e-6 * max(abs(fd), 1.0)


def test_wendland_c2_kernel(orc):
    # The Wendland C2 variant: normalised over the unit support, zero value
    # and slope at the edge, zero slope at the origin, derivative against a
    # central difference; and for both kernels H / h = 1 / (2 sigma) with
    # sigma the per-axis standard deviation of the unit-support kernel,
    # which fixes the two gamma_k constants (1.825742 for M4, 1.936492 for
    # C2) from the kernel shapes alone.
    k = "wendland_c2"
    val, _ = integrate.quad(lambda u: 4.0 * math.pi * u * u * orc.w_hat(u, k), 0.0, 1.0,
                            epsabs=1e-14, epsrel=1e-14)
    assert abs(val - 1.0) < 1e-12
    assert orc.w_hat(1.0, k) == 0.0 and orc.dw_hat(1.0, k) == 0.0 and orc.dw_hat(0.0, k) == 0.0
    assert orc.w_hat(1.2, k) == 0.0 and abs(orc.dw_hat(1.0 - 1e-6, k)) < 1e-15
    for u in np.linspace(0.01, 0.99, 99):
        d = 1e-6
        fd = (orc.w_hat(u + d, k) - orc.w_hat(u - d, k)) / (2 * d)
        assert abs(fd - orc.dw_hat(u, k)) < 1e-7 * max(1.0, abs(fd))
    for kern, g in (("m4", orc.GAMMA_K), (k, orc.GAMMA_K_WENDLAND_C2)):
        m2, _ = integrate.quad(lambda u: 4.0 * math.pi * u ** 4 * orc.w_hat(u, kern), 0.0, 1.0,
                               points=[0.5], epsabs=1e-15, epsrel=1e-14)
        assert abs(1.0 / (2.0 * math.sqrt(m2 / 3.0)) - g) < 1e-6, kern


@pytest.mark.parametrize("kernel", ["m4", "wendland_c2"])
def test_lattice_and_conservation_per_kernel(orc, kernel):
    # Both kernels: the perfect-lattice density equals the direct lattice
    # sum of the kernel (independent of the cell list), the lattice at rest
    # feels no force, and a jittered set conserves momentum and energy.
    prm = orc.params(kernel=kernel)
    ps = inputs.lattice_set(16, 0, perfect=True, order="shuffled")
    a = prm.gamma_k * inputs.ETA
    K = int(math.ceil(a)) + 1
    r = np.arange(-K, K + 1)
    kx, ky, kz = np.meshgrid(r, r, r, indexing="ij")
    dist = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2).ravel()
    dist = dist[dist < a]
    S = sum(orc.w_hat(t / a, kernel) for t in dist)
    d = orc.density(ps, prm, n_c=4)
    assert np.all(d["nngb"] == len(dist))
    assert np.max(np.abs(d["rho"] * a ** 3 / S - 1.0)) < 1e-13
    assert np.max(np.abs(d["wcount"] - 4.0 * math.pi / 3.0 * S)) < 1e-11
    f = orc.force(ps, d, prm, n_c=4)
    assert np.max(np.abs(f["a"])) < 1e-7 and np.max(np.abs(f["du"])) == 0.0
    js = inputs.small_set(1)
    d = orc.density(js, prm, n_c=4)
    f = orc.force(js, d, prm, n_c=4)
    red = orc.reduce(js.m, js.v, f["a"], f["du"])
    assert np.linalg.norm(red[:3]) / red[4] <= 1e-12 and abs(red[3]) / red[5] <= 1e-12
    assert red[4] > 1e-3
    db = orc.density(js, prm, mode="brute")
    assert all(np.array_equal(db[q], d[q]) for q in d)


def test_neighbour_number_convention(orc):
    # (4 pi / 3)(gamma_k eta)^3 ~ 48 neighbours at eta = 1.2348: pins the
    # H = gamma_k h convention (H = 2h would give ~63).
    n = 4.0 * math.pi / 3.0 * (orc.GAMMA_K * inputs.ETA) ** 3
    assert abs(n - 48.0) < 0.01


# --------------------------------------------------------------------------
# Perfect lattice closed form (Eq. density on a cubic lattice)
# --------------------------------------------------------------------------

def _lattice_sums(orc, a):
    """Direct sums over lattice vectors k in Z^3 with |k| < a (spacing 1):
    rho * a^3 = sum w_hat(|k|/a), n = #k, and d/da of rho."""
    K = int(math.ceil(a)) + 1
    r = np.arange(-K, K + 1)
    kx, ky, kz = np.meshgrid(r, r, r, indexing="ij")
    d = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2).ravel()
    d = d[d < a]
    S = sum(orc.w_hat(t / a) for t in d)
    return S, len(d)


@pytest.mark.parametrize("n_side,n_c,mode", [(8, 3, "brute"), (16, 4, "cells"), (16, 4, "brute")])
def test_perfect_lattice_closed_form(orc, n_side, n_c, mode):
    # rho = a^-3 sum_k w_hat(|k|/a) with a = gamma_k eta, independent of the
    # periodic box, the cell list and the particle order; a = du = 0 at rest.
    ps = inputs.lattice_set(n_side, 0, perfect=True, order="shuffled")
    a = orc.GAMMA_K * inputs.ETA
    S, nk = _lattice_sums(orc, a)
    rho_cf = S / a ** 3
    d = orc.density(ps, mode=mode, n_c=n_c)
    assert np.all(d["nngb"] == nk) and nk == 57
    assert np.max(np.abs(d["rho"] / rho_cf - 1.0)) < 1e-13
    assert abs(rho_cf - 1.0039808) < 5e-8
    assert np.max(np.abs(d["wcount"] - 4.0 * math.pi / 3.0 * S)) < 1e-11
    # d rho / d h on the lattice: rho(a) scales as a^-3 S(a); FD in a
    da = 1e-6 * a
    drho_da = ((_lattice_sums(orc, a + da)[0] / (a + da) ** 3) -
               (_lattice_sums(orc, a - da)[0] / (a - da) ** 3)) / (2 * da)
    # h = a dx / gamma_k  =>  h/(3 rho) d rho/dh = a/(3 rho) d rho/da
    want = a / (3.0 * rho_cf) * drho_da
    got = ps.h[0] * d["rho_dh"] / (3.0 * d["rho"])
    assert np.max(np.abs(got - want)) < 1e-7
    f = orc.force(ps, d, mode=mode, n_c=n_c)
    assert np.max(np.abs(f["a"])) < 1e-10 * 1e3
    assert np.max(np.abs(f["du"])) == 0.0


# --------------------------------------------------------------------------
# Brute force == cell list, bit for bit (the cell list only restricts the
# candidates; every sum runs over the same ascending neighbour list)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small(orc):
    ps = inputs.small_set(1, order="shuffled")
    return ps


def test_brute_equals_cells(orc, small):
    db = orc.density(small, mode="brute")
    dc = orc.density(small, mode="cells", n_c=4)
    for k in db:
        assert np.array_equal(db[k], dc[k]), k
    fb = orc.force(small, db, mode="brute")
    fc = orc.force(small, dc, mode="cells", n_c=4)
    for k in fb:
        assert np.array_equal(fb[k], fc[k]), k
    n1 = orc.near_support(small, 4, mode="brute", eps_rel=1e-3)
    n2 = orc.near_support(small, 4, mode="cells", eps_rel=1e-3)
    assert np.array_equal(n1[0], n2[0]) and np.array_equal(n1[1], n2[1])
    assert n1[1].sum() > 0


def test_cell_list_rejects_small_cells(orc, small):
    with pytest.raises(ValueError):
        orc.density(small, mode="cells", n_c=8)     # side 1/8 < H


# --------------------------------------------------------------------------
# Conservation (pairwise antisymmetry of Eq. momentum; energy balance)
# --------------------------------------------------------------------------

def test_momentum_and_energy_conservation(orc, small):
    d = orc.density(small, n_c=4)
    f = orc.force(small, d, n_c=4)
    r = orc.reduce(small.m, small.v, f["a"], f["du"])
    assert np.linalg.norm(r[:3]) / r[4] <= 1e-12
    assert abs(r[3]) / r[5] <= 1e-12
    # forces are not trivially zero on the jittered lattice
    assert r[4] > 1e-3


def test_conservation_with_uneven_h(orc, small):
    # Uneven h makes g_i != g_j, so a viscosity or pressure term that uses
    # one side's kernel gradient only breaks the pairwise antisymmetry.
    rng = np.random.default_rng(9)
    ps = inputs.ParticleSet(small.x, small.v * 30.0, small.m * rng.uniform(0.5, 1.5, small.n),
                            small.h * rng.uniform(0.7, 1.0, small.n),
                            small.u * rng.uniform(0.5, 2.0, small.n))
    d = orc.density(ps, n_c=4)
    f = orc.force(ps, d, n_c=4)
    r = orc.reduce(ps.m, ps.v, f["a"], f["du"])
    assert np.linalg.norm(r[:3]) / r[4] <= 1e-12
    assert abs(r[3]) / r[5] <= 1e-12


def test_galilean_invariance(orc, small):
    d = orc.density(small, n_c=4)
    f0 = orc.force(small, d, n_c=4)
    boosted = inputs.ParticleSet(small.x, small.v + np.array([0.3, -0.2, 0.1]), small.m,
                                 small.h, small.u)
    f1 = orc.force(boosted, d, n_c=4)
    scale = np.abs(f0["a"]).mean()
    assert np.max(np.abs(f1["a"] - f0["a"])) <= 1e-12 * scale * 1e3
    assert np.max(np.abs(f1["du"] - f0["du"])) <= 1e-12 * np.abs(f0["du"]).mean() * 1e3


def test_density_dh_finite_difference_on_jittered_set(orc, small):
    # d rho_i / d h_i against a central difference of rho_i(h_i): rho_i
    # depends only on h_i, so scaling every h probes every particle.
    d0 = orc.density(small, n_c=4)
    eps = 1e-6
    sp = inputs.ParticleSet(small.x, small.v, small.m, small.h * (1 + eps), small.u)
    sm = inputs.ParticleSet(small.x, small.v, small.m, small.h * (1 - eps), small.u)
    rp = orc.density(sp, n_c=4)["rho"]
    rm = orc.density(sm, n_c=4)["rho"]
    fd = (rp - rm) / (2 * eps * small.h)
    scale = np.abs(d0["rho"] / small.h)
    assert np.max(np.abs(fd - d0["rho_dh"]) / scale) < 1e-6


def test_gradh_off_reduces_to_printed_momentum_equation(orc):
    # With f = 1 and uniform h, the force loop is Eq. momentum as printed:
    # dv_i/dt = -sum_j m_j (P_i/rho_i^2 + P_j/rho_j^2) grad_i W(r_ij, h)
    # (no viscosity: alpha = 0). Direct numpy sum over all pairs.
    ps = inputs.lattice_set(8, 3, order="shuffled")
    prm = orc.params(alpha=0.0, gradh=False)
    d = orc.density(ps, prm, mode="brute")
    f = orc.force(ps, d, prm, mode="brute")
    x = ps.x
    dd = x[:, None, :] - x[None, :, :]
    dd -= np.rint(dd)
    r = np.sqrt((dd ** 2).sum(-1))
    H = orc.GAMMA_K * ps.h[0]
    np.fill_diagonal(r, 1.0)
    u = r / H
    dw = np.vectorize(orc.dw_hat)(u) / H ** 4
    dw[u >= 1.0] = 0.0
    np.fill_diagonal(dw, 0.0)
    Pr = d["P"] / d["rho"] ** 2
    coef = ps.m[None, :] * (Pr[:, None] + Pr[None, :]) * dw / r
    a_ref = -(coef[:, :, None] * dd).sum(1)
    assert np.max(np.abs(a_ref - f["a"])) <= 1e-10 * np.abs(a_ref).max()


def test_viscosity_two_body(orc):
    # Pressureless pair (u = 0): receding particles feel nothing; approaching
    # ones are pushed apart and heated, with kinetic energy turned into heat.
    base = dict(m=np.full(2, 0.5), h=np.full(2, 0.05), u=np.zeros(2))
    x = np.array([[0.50, 0.5, 0.5], [0.56, 0.5, 0.5]])
    for sign in (+1, -1):
        v = np.array([[-0.1 * sign, 0, 0], [0.1 * sign, 0, 0]])
        ps = inputs.ParticleSet(x, v, **base)
        d = orc.density(ps, mode="brute")
        f = orc.force(ps, d, mode="brute")
        if sign > 0:      # receding
            assert np.all(f["a"] == 0.0) and np.all(f["du"] == 0.0)
        else:             # approaching: particle 0 pushed to -x, 1 to +x
            assert f["a"][0, 0] < 0 < f["a"][1, 0]
            assert np.all(f["du"] > 0)
            dke = (ps.m[:, None] * v * f["a"]).sum()
            assert dke < 0 and abs(dke + (ps.m * f["du"]).sum()) < 1e-12 * abs(dke)
            assert abs(f["a"][0, 0] + f["a"][1, 0]) < 1e-12 * abs(f["a"][0, 0])


# --------------------------------------------------------------------------
# Variational pin of the grad-h force and the energy equation.
# With h_i = eta (m_i / rho_i)^(1/3) solved self-consistently and an
# adiabatic gas u_i = K_i rho_i^(gamma-1) / (gamma-1), the pressure force is
#   m_i dv_i/dt = -dE/dx_i,  E = sum_j m_j u_j,
# and du_i/dt is the time derivative of u_i along x + v t. Both sides are
# computed from rho alone, so f_i, A_i, g_i, g_j, the pair direction and the
# energy term are all checked without restating the force expression.
# --------------------------------------------------------------------------

def _solve_h(orc, ps, prm, eta=inputs.ETA, iters=60):
    h = ps.h.copy()
    for _ in range(iters):
        q = inputs.ParticleSet(ps.x, ps.v, ps.m, h, ps.u)
        d = orc.density(q, prm, mode="brute")
        F = d["rho"] * h ** 3 - ps.m * eta ** 3
        dF = d["rho_dh"] * h ** 3 + 3 * d["rho"] * h ** 2
        step = F / dF
        h = h - step
        if np.max(np.abs(step / h)) < 1e-15:
            break
    q = inputs.ParticleSet(ps.x, ps.v, ps.m, h, ps.u)
    return q, orc.density(q, prm, mode="brute")


@pytest.mark.parametrize("kernel", ["m4", "wendland_c2"])
def test_gradh_force_is_energy_gradient(orc, kernel):
    gam = 5.0 / 3.0
    prm = orc.params(alpha=0.0, kernel=kernel)
    ps0 = inputs.lattice_set(6, 11, jitter=0.15, order="shuffled")
    rng = np.random.default_rng(5)
    ps0.m = ps0.m * rng.uniform(0.7, 1.3, ps0.n)        # uneven masses -> uneven h
    ps, d = _solve_h(orc, ps0, prm)
    Kent = (gam - 1.0) * ps.u / d["rho"] ** (gam - 1.0)    # entropy, fixed

    def energy(x):
        q, dq = _solve_h(orc, inputs.ParticleSet(x, ps.v, ps.m, ps.h, ps.u), prm)
        uq = Kent * dq["rho"] ** (gam - 1.0) / (gam - 1.0)
        return float((ps.m * uq).sum())

    f = orc.force(ps, d, prm, mode="brute")
    for i in (0, 7, 100):
        for k in range(3):
            delta = 1e-6
            xp, xm = ps.x.copy(), ps.x.copy()
            xp[i, k] += delta
            xm[i, k] -= delta
            dE = (energy(xp) - energy(xm)) / (2 * delta)
            want = -dE / ps.m[i]
            assert abs(f["a"][i, k] - want) <= 2e-6 * np.abs(f["a"][i]).max(), (i, k)

    # du_i/dt = d/dt u_i(rho_i(x + v t)) along the adiabat
    def u_at(t):
        q, dq = _solve_h(orc, inputs.ParticleSet(ps.x + ps.v * t, ps.v, ps.m, ps.h, ps.u), prm)
        return Kent * dq["rho"] ** (gam - 1.0) / (gam - 1.0)

    dt = 1e-4
    du_fd = (u_at(dt) - u_at(-dt)) / (2 * dt)
    assert np.max(np.abs(du_fd - f["du"])) <= 1e-6 * np.abs(f["du"]).max()


# --------------------------------------------------------------------------
# Binning
# --------------------------------------------------------------------------

def test_binning_definition(orc):
    rng = np.random.default_rng(3)
    x = rng.uniform(-0.5, 1.5, size=(5000, 3))
    x[:5] = [[0.0, 0, 0], [1.0, 0.25, 0.5], [-1e-18, 0.3, 0.999999999999999],
             [0.75, 0.75, 0.75], [1 - 1e-17, 0.5, 0.5]]
    n_c = 4
    cell, start, perm, off = orc.bin_cells(x, n_c)
    xw = x - np.floor(x)
    c3 = np.minimum(np.floor(xw * n_c).astype(int), n_c - 1)
    assert np.array_equal(cell, c3[:, 0] + n_c * (c3[:, 1] + n_c * c3[:, 2]))
    # stable order by (cell, index): numpy's lexsort is the reference
    assert np.array_equal(perm, np.lexsort((np.arange(len(x)), cell)))
    assert np.array_equal(start, np.searchsorted(np.sort(cell), np.arange(n_c ** 3 + 1)))
    assert np.all(off >= 0.0) and np.all(off <= 1.0 / n_c)
    assert np.array_equal(off, xw - c3 / n_c)


def test_near_support_closed_forms(orc):
    """Pairs near a support radius: none on the perfect lattice (its shells
    lie at sqrt(5) and sqrt(6) spacings, the support at 2.254); for two
    particles at separation H (1 + t) the pair is near exactly when
    |t| H < eps_rel H + eps_abs, in both lists; in the force list a pair is
    near when it is near either particle's support."""
    lat = inputs.lattice_set(16, 0, perfect=True, order="shuffled")
    nd, nf = orc.near_support(lat, 4)
    assert not nd.any() and not nf.any()
    h = 0.05
    H = orc.GAMMA_K * h
    for t, want in ((1e-7, 1), (-4e-6, 1), (3e-5, 0), (-2e-3, 0)):
        x = np.array([[0.5, 0.5, 0.5], [0.5 + H * (1 + t), 0.5, 0.5]])
        ps = inputs.ParticleSet(x, np.zeros((2, 3)), np.ones(2), np.full(2, h), np.ones(2))
        nd, nf = orc.near_support(ps, 3, mode="brute", eps_rel=1e-5, eps_abs=0.0)
        assert nd.tolist() == [want, want] and nf.tolist() == [want, want], t
    # H_j > H_i: the pair sits at H_j only, so it is near in the force list of
    # both particles and in the density list of j alone
    x = np.array([[0.5, 0.5, 0.5], [0.5 + 2 * H, 0.5, 0.5]])
    ps = inputs.ParticleSet(x, np.zeros((2, 3)), np.ones(2), np.array([h, 2 * h]), np.ones(2))
    nd, nf = orc.near_support(ps, 3, mode="brute", eps_rel=1e-5, eps_abs=0.0)
    assert nd.tolist() == [0, 1] and nf.tolist() == [1, 1]


def test_fp32_counts_equal_fp64_counts_away_from_the_boundary(orc):
    """A neighbour count whose support test is taken in FP32 (here numpy's
    plain float32 arithmetic on the FP32 cell offsets, an order unrelated to
    the kernels') equals the FP64 brute-force count for every particle with
    no pair near a support radius, and differs by at most the number of
    such pairs for the others; those are a small fraction."""
    for ps, n_c in ((inputs.small_set(1), 4), (inputs.clustered_set(4000, 7, f_blob=0.4,
                                                                     sigma=0.05), None)):
        ps = ps.rounded_to("f32")
        if n_c is None:
            n_c = int(np.floor(1.0 / (orc.GAMMA_K * ps.h.max())))
        d = orc.density(ps, mode="brute")
        f = orc.force(ps, d, mode="brute")
        near_d, near_f = orc.near_support(ps, n_c)
        cell, _, _, off = orc.bin_cells(ps.x, n_c)
        c3 = np.stack([cell % n_c, (cell // n_c) % n_c, cell // (n_c * n_c)], 1)
        o32 = off.astype(np.float32)
        s = np.float32(1.0 / n_c)
        H32 = np.float32(orc.GAMMA_K) * ps.h.astype(np.float32)
        nd = np.zeros(ps.n, np.int64)
        nf = np.zeros(ps.n, np.int64)
        for i in range(ps.n):
            dc = c3 - c3[i]
            dc -= n_c * np.rint(dc / n_c).astype(np.int64)       # periodic cell separation
            ok = np.all(np.abs(dc) <= 1, axis=1)
            rel = (o32[ok] + dc[ok].astype(np.float32) * s) - o32[i]
            r2 = (rel * rel).sum(1, dtype=np.float32)
            hi2, hj2 = H32[i] * H32[i], H32[ok] * H32[ok]
            nd[i] = np.count_nonzero(r2 < hi2)
            nf[i] = np.count_nonzero((r2 < np.maximum(hi2, hj2)) & (np.nonzero(ok)[0] != i))
        clear_d, clear_f = near_d == 0, near_f == 0
        assert np.array_equal(nd[clear_d], d["nngb"][clear_d])
        assert np.array_equal(nf[clear_f], f["nforce"][clear_f])
        assert np.all(np.abs(nd - d["nngb"]) <= near_d)
        assert np.all(np.abs(nf - f["nforce"]) <= near_f)
        assert clear_d.mean() > 0.99 and clear_f.mean() > 0.98


# --------------------------------------------------------------------------
# Kick / drift (Alg. 1 CallLinear)
# --------------------------------------------------------------------------

def test_kick_drift_special_cases(orc):
    x = np.array([[0.99, 0.5, 0.01], [0.2, 0.2, 0.2]])
    v = np.array([[0.2, 0.0, -0.2], [0.0, 0.0, 0.0]])
    u = np.array([1.0, 2.0])
    a = np.array([[0.0, 0.0, 0.0], [1.0, -2.0, 0.5]])
    du = np.array([0.0, -1.0])
    xn, vn, un = orc.kick_drift(x, v, u, a, du, 0.1, 0.1)
    assert np.array_equal(vn[0], v[0]) and un[0] == 1.0        # no acceleration
    assert np.all((xn >= 0) & (xn < 1))                        # wrapped
    assert abs(xn[0, 0] - 0.01) < 1e-15 and abs(xn[0, 2] - 0.99) < 1e-15
    assert np.allclose(vn[1], [0.1, -0.2, 0.05], rtol=0, atol=1e-16)
    assert np.allclose(xn[1], [0.21, 0.18, 0.205], rtol=0, atol=1e-16)  # drift uses kicked v
    assert abs(un[1] - 1.9) < 1e-15


# --------------------------------------------------------------------------
# Quantisers (Sec. 3.2, Table 2): library routines as references
# --------------------------------------------------------------------------

def test_table2_formats(orc):
    g = json.load(open(os.path.join(GOLDEN, "table2_formats.json")))["formats"]
    f16 = g["f16"]
    # smallest normal, machine epsilon and largest finite value of the half
    # layout follow from 5 exponent and 10 mantissa bits
    emax = 2 ** (f16["exponent"] - 1) - 1
    assert orc.roundtrip(2.0 ** (1 - emax), "f16") == 2.0 ** (1 - emax)
    assert orc.roundtrip(1 + 2.0 ** -f16["mantissa"], "f16") == 1 + 2.0 ** -f16["mantissa"]
    assert orc.roundtrip(1 + 2.0 ** -(f16["mantissa"] + 1), "f16") == 1.0
    big = (2 - 2.0 ** -f16["mantissa"]) * 2.0 ** emax
    assert orc.roundtrip(big, "f16") == big
    assert math.isinf(orc.roundtrip(2.0 ** (emax + 1), "f16"))
    f32 = g["f32"]
    assert orc.roundtrip(1 + 2.0 ** -f32["mantissa"], "f32") == 1 + 2.0 ** -f32["mantissa"]
    assert orc.roundtrip(1 + 2.0 ** -(f32["mantissa"] + 1), "f32") == 1.0
    # bfloat16: single's 8-bit exponent, 7 mantissa bits
    assert orc.roundtrip(1 + 2.0 ** -7, "bf16") == 1 + 2.0 ** -7
    assert orc.roundtrip(1 + 2.0 ** -8, "bf16") == 1.0
    assert orc.roundtrip(2.0 ** -126, "bf16") == 2.0 ** -126


def _all_f32_chunks(chunk=1 << 26):
    """Every FP32 bit pattern when SPH_EXHAUSTIVE=1 (about 7 minutes for both
    formats); otherwise every 61st pattern plus every pattern whose upper 16
    bits are one of a spread of exponents (all rounding cases of those)."""
    if os.environ.get("SPH_EXHAUSTIVE") == "1":
        for start in range(0, 1 << 32, chunk):
            yield np.arange(start, start + chunk, dtype=np.uint64).astype(np.uint32).view(np.float32)
        return
    yield np.arange(0, 1 << 32, 61, dtype=np.uint64).astype(np.uint32).view(np.float32)
    low = np.arange(1 << 16, dtype=np.uint32)
    for hi in (0x0000, 0x3300, 0x3380, 0x3880, 0x3f80, 0x4780, 0x477f, 0x7f7f, 0x7f80,
               0x8000, 0xb380, 0xc77f, 0xff80):
        yield ((np.uint32(hi) << np.uint32(16)) | low).view(np.float32)


def test_f16_quantiser_exhaustive(orc):
    # every FP32 bit pattern against numpy's IEEE float32 -> float16 cast
    for a in _all_f32_chunks():
        got = orc.quant(a, "f16")
        with np.errstate(over="ignore", invalid="ignore"):
            ref = a.astype(np.float16).view(np.uint16)
        nan = np.isnan(a)
        assert np.array_equal(got[~nan], ref[~nan])
        assert np.all((got[nan] & 0x7c00) == 0x7c00) and np.all(got[nan] & 0x3ff)
        back = orc.dequant(got[~nan], "f16")
        assert np.array_equal(back.view(np.uint32), ref[~nan].view(np.float16)
                              .astype(np.float32).view(np.uint32))


def test_bf16_quantiser_exhaustive(orc):
    torch = pytest.importorskip("torch")
    for a in _all_f32_chunks():
        got = orc.quant(a, "bf16")
        ref = torch.from_numpy(a).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
        nan = np.isnan(a)
        assert np.array_equal(got[~nan], ref[~nan])
        assert np.all((got[nan] & 0x7f80) == 0x7f80) and np.all(got[nan] & 0x7f)
        back = orc.dequant(got[~nan], "bf16")
        assert np.array_equal(back, torch.from_numpy(ref[~nan].view(np.int16))
                              .view(torch.bfloat16).float().numpy())


def test_dequantise_set_roundtrips(orc, small):
    q = orc.dequantise_set(small, 4, pos="f16", vel="bf16", mhu="f16", scales=(12, 3, 0))
    cell, start, perm, off = orc.bin_cells(small.x, 4)
    c3 = np.stack([cell % 4, (cell // 4) % 4, cell // 16], 1)
    off16 = off.astype(np.float32).astype(np.float16).astype(np.float64)
    assert np.array_equal(q.x, c3 / 4.0 + off16)
    m16 = (small.m * 2 ** 12).astype(np.float32).astype(np.float16).astype(np.float64)
    assert np.array_equal(q.m, m16 / 2 ** 12)
    h16 = (small.h * 2 ** 3).astype(np.float32).astype(np.float16).astype(np.float64)
    assert np.array_equal(q.h, h16 / 2 ** 3)
    assert np.array_equal(q.u, small.u.astype(np.float32).astype(np.float16).astype(np.float64))


@pytest.mark.parametrize("n_c,bits", [(4, 0), (4, 1), (5, 2), (3, 3)])
def test_sub_cell_order(orc, n_c, bits):
    # key = cell * R^3 + Morton(sub-cell); perm is numpy's stable lexsort by
    # (key, index); sub_start is the CSR of the keys; bits = 0 is the plain
    # cell order
    rng = np.random.default_rng(n_c * 10 + bits)
    x = rng.uniform(-0.2, 1.2, size=(3000, 3))
    x[:3] = [[0.0, 0.0, 0.0], [1 - 1e-17, 0.5, 0.5], [0.25, 0.5, 0.75]]
    key, start, perm = orc.bin_sub(x, n_c, bits)
    R = 1 << bits
    xw = x - np.floor(x)
    c3 = np.minimum(np.floor(xw * n_c).astype(int), n_c - 1)
    s3 = np.clip(np.floor(xw * (n_c * R)).astype(int) - c3 * R, 0, R - 1)
    mort = np.zeros(len(x), np.int64)
    for b in range(bits):
        for a in range(3):
            mort |= ((s3[:, a] >> b) & 1) << (3 * b + a)
    cell = c3[:, 0] + n_c * (c3[:, 1] + n_c * c3[:, 2])
    assert np.array_equal(key, cell * R ** 3 + mort)
    assert np.array_equal(perm, np.lexsort((np.arange(len(x)), key)))
    assert np.array_equal(start, np.searchsorted(np.sort(key), np.arange(n_c ** 3 * R ** 3 + 1)))
    if bits == 0:
        assert np.array_equal(perm, orc.bin_cells(x, n_c)[2])
    # particles of one sub-cell lie inside its box
    side = 1.0 / (n_c * R)
    assert np.all(xw >= (c3 * R + s3) * side - 1e-15)


def test_cell_pair_partials_partition_the_full_sums(orc):
    """Restricting j to one neighbour cell (a serving task) splits each sum:
    over the 27 cells around i's cell the partial counts add up exactly to
    the full counts (brute force), and the partial rho, a, du to the full
    values within FP64 summation rounding; vsig is the max of the partial
    maxima."""
    ps = inputs.clustered_set(3000, 11, f_blob=0.4, sigma=0.06)
    n_c = int(np.floor(1.0 / (orc.GAMMA_K * ps.h.max())))
    assert n_c >= 3
    dens = orc.density(ps, mode="brute")
    full_f = orc.force(ps, dens, mode="brute")
    cell, start, perm, _ = orc.bin_cells(ps.x, n_c)
    rng = np.random.default_rng(5)
    cells = rng.choice(np.nonzero(np.diff(start) > 0)[0], size=6, replace=False)
    for ci in cells:
        cx, cy, cz = ci % n_c, (ci // n_c) % n_c, ci // (n_c * n_c)
        nbr = sorted({((cx + dx) % n_c) + n_c * (((cy + dy) % n_c) + n_c * ((cz + dz) % n_c))
                      for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)})
        tasks = [(k, ci, cj, start[ci], start[ci + 1]) for k in (0, 1) for cj in nbr]
        parts = orc.task_partials(ps, n_c, tasks, dens, perm=perm, cell=cell)
        idx = perm[start[ci]:start[ci + 1]]
        dp = [p for t, p in zip(tasks, parts) if t[0] == 0]
        fp = [p for t, p in zip(tasks, parts) if t[0] == 1]
        assert np.array_equal(sum(p["count"] for p in dp), dens["nngb"][idx])
        assert np.array_equal(sum(p["count"] for p in fp), full_f["nforce"][idx])
        np.testing.assert_allclose(sum(p["rho"] for p in dp), dens["rho"][idx], rtol=1e-13)
        np.testing.assert_allclose(sum(p["rho_dh"] for p in dp), dens["rho_dh"][idx],
                                   rtol=1e-12, atol=1e-12 * np.abs(dens["rho_dh"]).max())
        asum = sum(p["a"] for p in fp)
        scale = np.abs(full_f["a"]).max()
        np.testing.assert_allclose(asum, full_f["a"][idx], rtol=0, atol=1e-12 * scale)
        np.testing.assert_allclose(sum(p["du"] for p in fp), full_f["du"][idx], rtol=0,
                                   atol=1e-12 * np.abs(full_f["du"]).max())
        vmax = np.max(np.stack([p["vsig"] for p in fp]), axis=0)
        assert np.array_equal(vmax, full_f["vsig"][idx])


def test_near_support_selection_is_a_subset(orc):
    """near_support over selected i returns exactly the full counts at those i."""
    ps = inputs.clustered_set(5000, 3, f_blob=0.4, sigma=0.06)
    n_c = int(np.floor(1.0 / (orc.GAMMA_K * ps.h.max())))
    nd, nf = orc.near_support(ps, n_c, eps_rel=1e-3)
    assert nf.sum() > 0
    sel = np.random.default_rng(2).choice(ps.n, 300, replace=False).astype(np.int32)
    a, b = orc.near_support(ps, n_c, sel=sel, eps_rel=1e-3)
    assert np.array_equal(a, nd[sel]) and np.array_equal(b, nf[sel])


def test_truncated_storage_formats(orc):
    """truncate_mantissa storage of T bits (Table 2): the IEEE sizes are the
    IEEE formats, other sizes keep the next wider layout's sign and exponent
    and cut its mantissa to T - 1 - e bits (toward zero)."""
    rng = np.random.default_rng(4)
    vals = np.concatenate([rng.normal(0, 1, 500), rng.uniform(-1e-3, 1e-3, 200),
                           [0.0, -0.0, 1.0, -2.5, 1e-30]])
    for v in vals:
        assert orc.roundtrip(v, "t64") == v
        assert orc.roundtrip(v, "t32") == orc.roundtrip(v, "f32")
        assert orc.roundtrip(v, "t16", 6) == orc.roundtrip(v, "f16", 6)
    # cut, not rounded: T = 40 (double layout, 28 mantissa bits), T = 20
    # (single layout, 11 bits), T = 12 (half layout, 6 bits)
    for T, m in (("t40", 28), ("t20", 11), ("t12", 6)):
        assert orc.roundtrip(1 + 2.0 ** -m, T) == 1 + 2.0 ** -m
        assert orc.roundtrip(1 + 2.0 ** -(m + 1), T) == 1.0
        assert orc.roundtrip(1 + 2.0 ** -m + 2.0 ** -(m + 1), T) == 1 + 2.0 ** -m
        assert orc.roundtrip(-(1 + 2.0 ** -(m + 1)), T) == -1.0
        assert orc.roundtrip(2 - 2.0 ** -(m + 1), T) == 2 - 2.0 ** -m
    # relative error of the cut: below 2^-m (plus the IEEE rounding to the base)
    for T in range(9, 64):
        e = 11 if T > 32 else (8 if T > 16 else 5)
        m = T - 1 - e
        base = 0.0 if T > 32 else (2.0 ** -24 if T > 16 else 2.0 ** -11 + 2.0 ** -24)
        for v in rng.uniform(0.5, 2.0, 50):
            q = orc.roundtrip(v, f"t{T}")
            assert abs(q) <= abs(v) * (1 + base)
            assert abs(q - v) <= (2.0 ** -m + base) * abs(v)


def test_truncation_error_curve_shape(orc):
    """Acceleration error of one force evaluation on truncated storage (all
    fields, T bits) against FP64, with FP64 arithmetic: zero at 64 bits,
    growing as bits are cut within each layout, and lower at exactly 32 and
    16 bits than one bit above, where the base layout switches to IEEE
    single and half (the shape the paper reports for its figure on the
    force kernel's error)."""
    ps = inputs.small_set(1)
    n_c = 4
    ref = inputs.unpack_aos(inputs.pack_aos(ps, "f64"))
    d0 = orc.density(ref, n_c=n_c)
    f0 = orc.force(ref, d0, n_c=n_c)
    e = {}
    for T in range(9, 65):
        q = orc.dequantise_set(ref, n_c, f"t{T}", f"t{T}", f"t{T}", (12, 3, 0))
        d = orc.density(q, n_c=n_c)
        f = orc.force(q, d, n_c=n_c)
        e[T] = np.sqrt((np.linalg.norm(f["a"] - f0["a"], axis=1) ** 2).mean()) / \
            np.linalg.norm(f0["a"], axis=1).mean()
    assert e[64] == 0.0
    for lo, hi in ((33, 63), (17, 31), (9, 15)):
        for T in range(lo, hi):
            assert e[T] > e[T + 1], T
    assert e[32] < e[33] and e[16] < e[17]


def test_smoothing_length_closed_forms(orc):
    """h = eta (m / rho(h))^(1/3): (1) with equal masses the weighted
    neighbour number at the root is (4 pi / 3) H^3 rho / m = (4 pi / 3)
    (gamma_k eta)^3 for every particle; (2) on a perfect lattice the root
    found by Newton steps equals the root of the direct lattice sum found by
    bisection; (3) brute force equals the cell list bit for bit; (4) a limit
    h_max below the root is kept and reported as not converged."""
    ps = inputs.small_set(4)
    n_c = 4
    h_max = 1.0 / (orc.GAMMA_K * n_c)
    start = ps.subset(np.arange(ps.n))
    start.h = ps.h * np.random.default_rng(1).uniform(0.7, 1.3, ps.n)
    h, it = orc.smoothing_length(start, n_c=n_c, tol=1e-10, max_iter=50)
    assert np.all(it <= 50)
    assert np.all(h < h_max)
    ph = ps.subset(np.arange(ps.n))
    ph.h = h
    d = orc.density(ph, n_c=n_c)
    target = 4.0 * np.pi / 3.0 * (orc.GAMMA_K * orc.ETA) ** 3
    np.testing.assert_allclose(d["wcount"], target, rtol=1e-8)
    hb, itb = orc.smoothing_length(start, n_c=n_c, tol=1e-10, max_iter=50, mode="brute")
    assert np.array_equal(h, hb) and np.array_equal(it, itb)
    # perfect lattice: bisection on rho(h) = m sum_k W(|k| a, h) from the pinned kernel
    n_side = 16
    a = 1.0 / n_side
    lat = inputs.lattice_set(n_side, 0, perfect=True)
    r = np.sqrt(((np.stack(np.meshgrid(*[np.arange(-4, 5)] * 3, indexing="ij"), -1)
                  .reshape(-1, 3) * a) ** 2).sum(1))
    rho = lambda hh: lat.m[0] * sum(orc.W(float(x), hh) for x in r)
    g = lambda hh: hh - orc.ETA * (lat.m[0] / rho(hh)) ** (1.0 / 3.0)
    lo, hi = 0.5 * orc.ETA * a, 1.5 * orc.ETA * a
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if g(mid) < 0 else (lo, mid)
    hl, _ = orc.smoothing_length(lat, n_c=n_c, tol=1e-12, max_iter=60, sel=np.arange(8))
    np.testing.assert_allclose(hl, 0.5 * (lo + hi), rtol=1e-10)
    # a limit below the root: kept, and the particle is reported unconverged
    h2, it2 = orc.smoothing_length(start, n_c=n_c, h_max=0.8 * ps.h.min(), tol=1e-8,
                                   max_iter=20, sel=np.arange(16))
    assert np.all(h2 == 0.8 * ps.h.min()) and np.all(it2 == 21)


# ---------------------------------------------------------------------------
# time integration: CFL step and leapfrog kick-drift-kick
# ---------------------------------------------------------------------------

def _moving_set(seed, v_sigma=0.3):
    ps = inputs.small_set(seed)
    ps.v = np.random.default_rng(seed).normal(0.0, v_sigma, ps.v.shape)
    return ps


def test_cfl_timestep_closed_form(orc):
    """Perfect lattice at rest: every signal velocity is 2c, so the step is
    c_cfl gamma_k h / (2 c), c = sqrt(gamma (gamma - 1) u); a particle with
    no neighbour (vsig = 0) sets no limit."""
    lat = inputs.lattice_set(16, 0, perfect=True)
    lat.v[:] = 0.0
    d = orc.density(lat, n_c=4)
    f = orc.force(lat, d, n_c=4)
    c = np.sqrt(orc.GAMMA * (orc.GAMMA - 1.0) * lat.u)
    np.testing.assert_allclose(f["vsig"], 2.0 * c, rtol=1e-14)
    dt, dmin = orc.timestep(lat.h, f["vsig"])
    np.testing.assert_allclose(dt, orc.C_CFL * orc.GAMMA_K * lat.h / (2.0 * c), rtol=1e-14)
    assert dmin == dt.min()
    dt2, dmin2 = orc.timestep(np.array([0.1, 0.2]), np.array([0.0, 4.0]))
    assert dt2[0] == np.inf and dmin2 == dt2[1] == orc.C_CFL * orc.GAMMA_K * 0.2 / 4.0


def test_kdk_energy_second_order(orc):
    """Total energy sum m (|v|^2 / 2 + u) is conserved by the equations;
    the leapfrog error over a fixed time falls with the square of the step
    (halving dt cuts it by about 4) without viscosity, where the flow is
    smooth. A first-order arrangement (forces taken with the half-step v
    and u instead of the predicted ones) only halves it. Momentum is
    conserved to rounding, viscosity included."""
    ps = _moving_set(22)
    for prm in (orc.params(alpha=0.0), orc.params()):
        err = {}
        for dt, n in ((4e-3, 6), (2e-3, 12), (1e-3, 24)):
            _, hist = orc.kdk_run(ps, 4, n, dt=dt, prm=prm)
            e = np.array([h["ekin"] + h["eth"] for h in hist])
            err[dt] = np.abs(e - e[0]).max() / e[0]
            p = np.array([h["p"] for h in hist])
            assert np.abs(p - p[0]).max() < 1e-13
        if prm.alpha == 0.0:
            assert 1e-8 < err[1e-3] < 1e-5, err
            assert 3.5 < err[4e-3] / err[2e-3] < 5.0, err
            assert 3.5 < err[2e-3] / err[1e-3] < 5.0, err
        else:
            # the viscosity switch min(w, 0) is not smooth: bounded and
            # falling with dt, but not by a clean power
            assert err[1e-3] < 1e-5 and err[4e-3] / err[1e-3] > 2.0, err
    # the same run with forces from the half-step v and u: first order
    prm = orc.params(alpha=0.0)
    err = {}
    for dt, n in ((2e-3, 12), (1e-3, 24)):
        x, v, u = ps.x.copy(), ps.v.copy(), ps.u.copy()
        at = lambda: inputs.ParticleSet(x, v, ps.m, ps.h, u)
        f = orc.force(at(), orc.density(at(), prm, n_c=4), prm, n_c=4)
        e0 = orc.totals(ps.m, v, u)
        for _ in range(n):
            x, v, u = orc.kick_drift(x, v, u, f["a"], f["du"], dt / 2, dt)
            f = orc.force(at(), orc.density(at(), prm, n_c=4), prm, n_c=4)
            x, v, u = orc.kick_drift(x, v, u, f["a"], f["du"], dt / 2, 0.0)
        e1 = orc.totals(ps.m, v, u)
        err[dt] = abs(e1["ekin"] + e1["eth"] - e0["ekin"] - e0["eth"])
    assert err[2e-3] / err[1e-3] < 2.5, err


def test_kdk_free_particles(orc):
    """Particles farther apart than their supports feel no force: x moves
    by v t exactly (modulo the box), v and u stay, and the CFL step sets no
    limit (no neighbour, vsig = 0)."""
    g = np.arange(4) / 4.0 + 0.125
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    n = x.shape[0]
    rng = np.random.default_rng(5)
    ps = inputs.ParticleSet(x, rng.normal(0, 0.5, (n, 3)), np.full(n, 1.0 / n),
                            np.full(n, 0.05), np.ones(n))
    out, hist = orc.kdk_run(ps, 4, 5, dt=0.01)
    want = ps.x + 0.05 * ps.v
    want -= np.floor(want)
    np.testing.assert_allclose(out.x, want, atol=1e-15)
    assert np.array_equal(out.v, ps.v) and np.array_equal(out.u, ps.u)
    f = orc.force(ps, orc.density(ps, n_c=4), n_c=4)
    assert np.all(f["vsig"] == 0.0) and orc.timestep(ps.h, f["vsig"])[1] == np.inf


# --------------------------------------------------------------------------
# Coincident positions and position anchors (reduced-precision storage)
# --------------------------------------------------------------------------

def test_coincident_pair_reading(orc):
    """Two particles j != i at the same position (reachable once positions
    are stored in FP16): the pair direction is the zero vector. The pair
    counts in both lists, exerts no force, does no work and has signal
    velocity c_i + c_j. This is the r -> 0 limit of the pair terms: the
    kernel gradient vanishes linearly at the origin, so the force of a pair
    at separation r falls to zero with r, and with v_i = v_j the signal
    velocity is c_i + c_j at every r."""
    h = 0.05
    res = {}
    for r in (0.0, 1e-9, 1e-7):
        x = np.array([[0.4, 0.5, 0.6], [0.4 + r, 0.5, 0.6], [0.4, 0.5 + 0.7 * h, 0.6]])
        v = np.array([[0.1, 0.0, 0.0], [0.1, 0.0, 0.0], [0.0, -0.2, 0.0]])
        ps = inputs.ParticleSet(x, v, np.full(3, 0.01), np.full(3, h), np.array([1.0, 2.0, 1.5]))
        d = orc.density(ps, mode="brute")
        f = orc.force(ps, d, mode="brute")
        assert np.all(np.isfinite(f["a"])) and np.all(np.isfinite(f["du"]))
        res[r] = (d, f)
    d0, f0 = res[0.0]
    assert d0["nngb"].tolist() == [3, 3, 3] and f0["nforce"].tolist() == [2, 2, 2]
    # continuity at r -> 0 of every output: the change is of order r / h (the
    # third particle interacts normally, its pair terms move with r too)
    for r in (1e-9, 1e-7):
        d1, f1 = res[r]
        for k in ("rho", "wcount", "rho_dh"):
            np.testing.assert_allclose(d1[k], d0[k], rtol=1e-10)
        scale = np.abs(f0["a"]).max()
        np.testing.assert_allclose(f1["a"], f0["a"], rtol=0, atol=10 * r / h * scale + 1e-15)
        np.testing.assert_allclose(f1["du"], f0["du"], rtol=0,
                                   atol=10 * r / h * np.abs(f0["du"]).max() + 1e-15)
        np.testing.assert_allclose(f1["vsig"], f0["vsig"], rtol=10 * r / h)
    # the coincident pair alone: no force, no heating, vsig = c_0 + c_1
    x = np.array([[0.4, 0.5, 0.6], [0.4, 0.5, 0.6]])
    ps = inputs.ParticleSet(x, np.array([[0.1, 0, 0], [-0.3, 0.2, 0]]), np.full(2, 0.01),
                            np.full(2, h), np.array([1.0, 2.0]))
    d = orc.density(ps, mode="brute")
    f = orc.force(ps, d, mode="brute")
    assert np.all(f["a"] == 0.0) and np.all(f["du"] == 0.0)
    c = np.sqrt(orc.GAMMA * (orc.GAMMA - 1) * ps.u)
    np.testing.assert_allclose(f["vsig"], [c.sum(), c.sum()], rtol=1e-15)
    assert f["nforce"].tolist() == [1, 1]


@pytest.mark.parametrize("anchor", [0, 1, 2, 3])
def test_position_anchors(orc, anchor):
    """Stored positions are offsets from an anchor (Sec. 3.2): the cell
    corner (0) or the centre of the particle's sub-cell of side
    1/(n_c 2^b) (1 + b). The anchor plus the FP64 offset gives back the
    wrapped position; the offset lies within half a sub-cell of the anchor
    (within the cell for the corner); the code holds the sub-cell indices;
    the FP16-stored position errs by at most half an FP16 ulp of that
    bound, so each level of anchor halves the worst error."""
    rng = np.random.default_rng(anchor + 40)
    n, n_c = 5000, 7
    x = rng.uniform(-0.3, 1.3, size=(n, 3))
    x[:4] = [[0, 0, 0], [1 - 1e-17, 0.5, 3 / 7], [2 / 7, 1 / 14, 0.999], [1 / 28, 3 / 28, 5 / 28]]
    off, code = orc.pos_offsets(x, n_c, anchor)
    xw = x - np.floor(x)
    c3 = np.minimum(np.floor(xw * n_c), n_c - 1)
    if anchor == 0:
        assert np.array_equal(off, orc.bin_cells(x, n_c)[3])
        assert not code.any()
        bound = 1.0 / n_c
        assert np.all(off >= 0) and np.all(off <= bound)
    else:
        R = 2 ** (anchor - 1)
        a3 = np.clip(np.floor(xw * n_c * R) - c3 * R, 0, R - 1)
        assert np.array_equal(code, (a3[:, 0] + 4 * a3[:, 1] + 16 * a3[:, 2]).astype(np.uint8))
        centre = (c3 * R + a3 + 0.5) / (n_c * R)
        np.testing.assert_array_equal(off, xw - centre)
        bound = 0.5 / (n_c * R)
        assert np.all(np.abs(off) <= bound * (1 + 1e-12))
    ps = inputs.ParticleSet(x, np.zeros((n, 3)), np.ones(n), np.ones(n), np.ones(n))
    q32 = orc.dequantise_set(ps, n_c, "f32", anchor=anchor)
    q16 = orc.dequantise_set(ps, n_c, "f16", anchor=anchor)
    assert np.max(np.abs(q32.x - xw)) <= 2.0 ** -24 * bound * (1 + 1e-9)
    e16 = np.max(np.abs(q16.x - xw))
    assert e16 <= 2.0 ** -11 * bound * (1 + 1e-9)
    assert e16 > 2.0 ** -13 * bound            # the bound is attained up to a factor 4
