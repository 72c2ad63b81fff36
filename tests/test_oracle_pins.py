"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks an oracle function against something other than itself:
numbers the paper prints (tests/golden/paper_values.json), closed forms,
library routines (scipy quad / spence / cKDTree), invariants and brute force.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, special
from scipy.spatial import cKDTree

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
ARCSEC = math.pi / 180 / 3600


# ------------------------------------------------------------- cosmology --
def test_lightcone_depth(orc):
    g = GOLD["lightcone_depth"]
    p = orc.default_params(Omega_m=g["Omega_m"])
    assert abs(orc.chi(p, g["z"]) / g["chi_mpch"] - 1) < g["rel_tol"]


def test_particle_mass_pins_rho_crit(orc):
    g = GOLD["particle_mass"]
    p = orc.default_params(Omega_m=g["Omega_m"])
    h = orc.solve_halo(p, 1e14, 5.0, 0.0)         # rho_crit at z = 0 in (Msun/h)/(Mpc/h)^3
    Mp = g["Omega_m"] * h.rho_crit * g["L_mpch"] ** 3 / g["N"] ** 3
    assert abs(Mp / g["M_p"] - 1) < g["rel_tol"]


@pytest.mark.parametrize("z", [0.1, 1.0, 3.0])
def test_einstein_de_sitter_closed_forms(orc, z):
    # Omega_m = 1: chi = 2 c/H0 (1 - 1/sqrt(1+z));  int (1+z)^2/E dz = (2/3)((1+z)^1.5 - 1)
    p = orc.default_params(Omega_m=1.0)
    cH = orc.C_CGS / 1e5 / 100.0
    assert abs(orc.chi(p, z) / (2 * cH * (1 - 1 / math.sqrt(1 + z))) - 1) < 1e-12
    H0 = 100 * p.h * 1e5 / orc.MPC
    rho_cr0 = 3 * H0 ** 2 / (8 * math.pi * orc.G_CGS)
    ne = p.Omega_b * rho_cr0 / (2 / (1 + p.X_H) * orc.M_P)
    tau_ref = orc.SIGMA_T * ne * orc.C_CGS / H0 * (2.0 / 3.0) * ((1 + z) ** 1.5 - 1)
    assert abs(orc.tau(p, z) / tau_ref - 1) < 1e-12
    assert abs(orc.D_A(p, z) * (1 + z) / orc.chi(p, z) - 1) < 1e-15


def test_tau_linear_in_omega_b(orc):
    p1, p2 = orc.default_params(Omega_b=0.04), orc.default_params(Omega_b=0.08)
    assert abs(orc.tau(p2, 1.0) / orc.tau(p1, 1.0) - 2) < 1e-13


# ---------------------------------------------------------- halo structure --
@pytest.mark.parametrize("x", [1e-6, 5e-5, 1e-4, 2e-4, 0.3, 1.0, 7.0, 30.0])
def test_m_nfw_is_integral(orc, x):
    ref = integrate.quad(lambda t: t / (1 + t) ** 2, 0, x, epsabs=0, epsrel=2e-14)[0]
    assert abs(orc.m_nfw(x) / ref - 1) < 1e-12


@pytest.mark.parametrize("x", [0.01, 0.3, 1.0, 3.0, 6.0])
def test_jeans_dispersion_closed_form(orc, x):
    # Lokas & Mamon closed form with Li2 against the Jeans-integral quadrature
    assert abs(orc.jeans_I(x) / orc.jeans_I(x, closed=True) - 1) < 1e-11


@pytest.mark.parametrize("x", [0.05, 0.5, 1.0, 2.0, 20.0])
def test_dilog(orc, x):
    assert abs(orc.li2_neg(x) - special.spence(1 + x)) < 1e-14 * max(1, abs(special.spence(1 + x)))
    assert abs(orc.li2_neg(1.0) + math.pi ** 2 / 12) < 1e-15


def test_jeans_equation_holds(orc, params):
    # d(rho sigma^2)/dr = -rho G M(r)/r^2 for the untruncated NFW halo
    h = orc.solve_halo(params, 1e14, 5.0, 0.3)
    rs = h.r_s * orc.MPC / params.h
    rho_s = h.rho_s * orc.MSUN / params.h / (orc.MPC / params.h) ** 3
    for x in (0.2, 1.0, 4.0):
        def p(xx):
            return rho_s / (xx * (1 + xx) ** 2) * orc.sigma2(params, h, xx)
        dx = 1e-4 * x
        dpdr = (p(x + dx) - p(x - dx)) / (2 * dx * rs)
        M = 4 * math.pi * rho_s * rs ** 3 * orc.m_nfw(x)
        rhs = -rho_s / (x * (1 + x) ** 2) * orc.G_CGS * M / (x * rs) ** 2
        assert abs(dpdr / rhs - 1) < 1e-6


CORNERS = [(10 ** 12.5, 2.0, 0.05), (10 ** 12.5, 15.0, 3.0), (10 ** 15.5, 2.0, 3.0), (10 ** 15.5, 15.0, 0.05),
           (1e14, 5.0, 0.5), (10 ** 12.5, 15.0, 0.05), (10 ** 15.5, 2.0, 0.05), (1e13, 6.0, 2.0)]


@pytest.mark.parametrize("M,c,z", CORNERS)
def test_halo_definitions(orc, params, M, c, z):
    h = orc.solve_halo(params, M, c, z)
    # virial radius definition and Delta_vir -> 18 pi^2 when Omega_m(z) -> 1
    assert abs(4 * math.pi / 3 * h.r_vir ** 3 * h.Delta_vir * h.rho_crit / M - 1) < 1e-13
    # r500: mean density inside is 500 rho_crit; M500 from the NFW enclosed mass
    assert abs(h.M500 / (4 * math.pi / 3 * h.r500 ** 3) / (500 * h.rho_crit) - 1) < 1e-10
    assert abs(h.M500 / M - orc.m_nfw(h.r500 / h.r_s) / orc.m_nfw(c)) < 1e-12
    # stellar mass and stellar radius: f_b M_tot(<r_*) = M_*
    fb = params.Omega_b / params.Omega_m
    assert abs(h.F_star - params.f_star * (h.M500 / params.h / 3e14) ** -params.S_star) < 1e-15
    assert abs(fb * M * orc.m_nfw(h.x_star) / orc.m_nfw(c) / h.M_star - 1) < 1e-11


def test_delta_vir_eds(orc):
    p = orc.default_params(Omega_m=1.0)
    h = orc.solve_halo(p, 1e14, 5.0, 1.0)
    assert abs(h.Delta_vir - 18 * math.pi ** 2) < 1e-12


@pytest.mark.parametrize("M,c,z", CORNERS[:4])
def test_initial_energy_closed_form(orc, params, M, c, z):
    h = orc.solve_halo(params, M, c, z)
    for xlo in (0.0, h.x_star):
        q, cl = orc.energy(params, h, xlo), orc.energy(params, h, xlo, closed=True)
        assert abs(q / cl - 1) < 1e-9
    fb = params.Omega_b / params.Omega_m
    assert abs(h.E_gi / (fb * orc.energy(params, h, h.x_star, closed=True)) - 1) < 1e-9
    assert h.E_gi < 0 and h.E_DM < 0


@pytest.mark.parametrize("M,c,z", CORNERS)
def test_boundary_conditions_solved(orc, params, M, c, z):
    h = orc.solve_halo(params, M, c, z)
    assert h.status == 0 and h.n_sign_changes == 1
    assert max(abs(h.res_M), abs(h.res_P), abs(h.res_E)) < 1e-10
    assert 0.9 < h.x_f < 2.6
    # the surface pressure is the pressure at r_f, from outside the solver
    P_s = params.Omega_b / params.Omega_m * h.rho_s / (c * (1 + c) ** 2) * \
        (orc.MSUN / params.h) / (orc.MPC / params.h) ** 3 * h.sigma2_vir
    assert abs(P_s / h.P_s - 1) < 1e-13
    # gas mass: integrate the gas density profile with scipy, independent of the solver
    X = params.X_H
    mu_e = 2 / (1 + X)
    u = orc.MPC / params.h

    def rho_g(r):
        return orc.profile(params, h, r)[1] * mu_e * orc.M_P
    pts = [h.r_vir] if h.r_vir < h.r_f else None
    Mgas = integrate.quad(lambda r: 4 * math.pi * (r * u) ** 2 * rho_g(r) * u, 0, h.r_f, points=pts,
                          epsabs=0, epsrel=1e-12, limit=200)[0]
    Mb = params.Omega_b / params.Omega_m * M * orc.MSUN / params.h
    assert abs((Mgas + h.M_star * orc.MSUN / params.h) / Mb - 1) < 1e-9
    # energy residual changes sign across the root
    assert orc.energy_residual_at(params, h, h.x_f * 0.99) * orc.energy_residual_at(params, h, h.x_f * 1.01) < 0


def test_energy_sign_reading_changes_root(orc):
    # the printed arrangement (energy_sign=1) puts r_f inside r_vir for low masses
    p1 = orc.default_params(energy_sign=1)
    h = orc.solve_halo(p1, 1e13, 5.0, 0.1)
    h0 = orc.solve_halo(orc.default_params(), 1e13, 5.0, 0.1)
    assert h.x_f < 0.8 < h0.x_f


def test_star_exceeds_baryons_flag(orc):
    p = orc.default_params(f_star=0.5)
    h = orc.solve_halo(p, 1e13, 5.0, 0.5)
    assert h.status == orc.NO_STAR_ROOT
    assert orc.solve_halo(orc.default_params(), -1.0, 5.0, 0.5).status == orc.BAD_INPUT


# ------------------------------------------------------- thermal & electrons --
def test_nonthermal_and_electron_factors(orc, params):
    g = GOLD["icm_table"]
    fmax = 4 ** -g["n_nt"] / g["alpha_nt"]
    assert abs(fmax - 1.8326499) < 1e-6
    assert orc.f_nt(params, 0.0) == 1.0
    assert abs(orc.f_nt(params, 60.0) - min(61 ** 0.5, (fmax - 1) * math.tanh(30) + 1)) < 1e-12
    h = orc.solve_halo(params, 1e14, 5.0, 0.5)
    X = GOLD["hydrogen_fraction"]["X"]
    Pe0, ne0 = orc.profile(params, h, 1e-12)
    assert abs(Pe0 / h.P0 - (2 * X + 2) / (5 * X + 3)) < 1e-9
    assert abs((2 * X + 2) / (5 * X + 3) - 0.5176470588) < 1e-9
    assert abs(ne0 * 2 / (1 + X) * orc.M_P / h.rho0 - 1) < 1e-9
    # electron pressure at r500 carries the (1 - R_nt) factor exactly
    r = h.r500
    Pe, _ = orc.profile(params, h, r)
    a = params.Gamma
    assert Pe > 0 and Pe < Pe0
    assert orc.profile(params, h, h.r_f * 1.0001) == (0.0, 0.0)
    assert h.R_t == min(h.r_f, 3 * h.r500)


# --------------------------------------------------------------- projection --
@pytest.mark.parametrize("frac", [0.0, 0.003, 0.4, 0.97, 1.02, 1.3])
def test_los_matches_brute_force(orc, params, frac):
    h = orc.solve_halo(params, 3e13, 6.0, 0.4)
    r = frac * h.r_vir
    if r >= h.r_f:
        assert orc.los(params, h, r) == (0.0, 0.0)
        return
    u = orc.MPC / params.h
    L = math.sqrt(h.r_f ** 2 - r ** 2)
    pts = [math.sqrt(h.r_vir ** 2 - r ** 2)] if r < h.r_vir < h.r_f else None
    ty, tb = orc.los(params, h, r)
    refy = 2 * integrate.quad(lambda l: orc.profile(params, h, math.hypot(r, l))[0], 0, L, points=pts,
                              epsabs=0, epsrel=1e-12, limit=400)[0] * u * orc.SIGMA_T / orc.ME_C2
    refb = 2 * integrate.quad(lambda l: orc.profile(params, h, math.hypot(r, l))[1], 0, L, points=pts,
                              epsabs=0, epsrel=1e-12, limit=400)[0] * u * orc.SIGMA_T
    assert abs(ty / refy - 1) < 1e-10 and abs(tb / refb - 1) < 1e-10


def test_projection_conserves_volume_integral(orc, params):
    # int Y(r_perp) 2 pi r_perp dr_perp over the disc = int P_e 4 pi r^2 dr over the sphere
    h = orc.solve_halo(params, 1e14, 4.0, 0.3)
    disc = integrate.quad(lambda r: orc.los(params, h, r)[0] * 2 * math.pi * r, 0, h.r_f,
                          points=[h.r_vir] if h.r_vir < h.r_f else None, epsabs=0, epsrel=1e-10, limit=200)[0]
    sph = integrate.quad(lambda r: orc.profile(params, h, r)[0] * 4 * math.pi * r * r, 0, h.r_f,
                         points=[h.r_vir] if h.r_vir < h.r_f else None, epsabs=0, epsrel=1e-12, limit=200)[0]
    u = orc.MPC / params.h
    assert abs(disc / (sph * u * orc.SIGMA_T / orc.ME_C2) - 1) < 1e-8


# -------------------------------------------------------------- HP flat map --
def test_hp_flat_conservation_and_sign(orc, params):
    # one halo well inside a small map: sum_p y dOmega = sigma_T/(m_e c^2) int_{cyl} P_e dV / D_A^2,
    # where the cylinder r_perp < R_t cuts the sphere; pixel-centre sampling error ~ 1e-4.
    h = orc.solve_halo(params, 2e14, 5.0, 0.3)
    npix = 96
    pix = 2.6 * h.R_t / h.D_A / npix
    cat = dict(M=[2e14], c=[5.0], z=[0.3], theta_x=[npix / 2 * pix + 0.3 * pix],
               theta_y=[npix / 2 * pix - 0.2 * pix], v_los=[250.0])
    y, b, halos = orc.hp_flat(params, cat, npix, pix)
    assert halos[0].status == 0
    tot = integrate.quad(lambda r: orc.los(params, h, r)[0] * 2 * math.pi * r, 0, h.R_t,
                         points=[h.r_vir] if h.r_vir < h.R_t else None, epsabs=0, epsrel=1e-10, limit=200)[0]
    Ymap = y.sum() * pix ** 2
    assert abs(Ymap / (tot / h.D_A ** 2) - 1) < 2e-3
    cat2 = dict(cat, v_los=[-250.0])
    y2, b2, _ = orc.hp_flat(params, cat2, npix, pix)
    assert np.array_equal(b2, -b) and np.array_equal(y2, y)
    # value at the pixel nearest the centre equals the direct LOS integral
    i, j = npix // 2, npix // 2 - 1
    dx, dy = (i + .5) * pix - cat["theta_x"][0], (j + .5) * pix - cat["theta_y"][0]
    assert abs(y[j, i] - orc.los(params, h, h.D_A * math.hypot(dx, dy))[0]) == 0.0


# ------------------------------------------------------------------ HEALPix --
@pytest.mark.parametrize("nside", [1, 2, 4, 8, 16])
def test_healpix_round_trip_and_rings(orc, nside):
    npix = 12 * nside * nside
    pix = np.arange(npix)
    th, ph = orc.pix2ang_ring(nside, pix)
    assert np.array_equal(orc.ang2pix_ring(nside, th, ph), pix)
    # ring structure: pixels with equal colatitude, 4i in caps and 4N in the belt
    rings = np.unique(np.round(np.cos(th), 12), return_counts=True)[1][::-1]
    expect = [4 * min(i, nside, 4 * nside - i) for i in range(1, 4 * nside)]
    assert list(rings) == expect
    assert np.all((ph >= 0) & (ph < 2 * math.pi))


def test_healpix_equal_area(orc):
    rng = np.random.default_rng(0)
    n = 200_000
    th = np.arccos(rng.uniform(-1, 1, n))
    ph = rng.uniform(0, 2 * math.pi, n)
    counts = np.bincount(orc.ang2pix_ring(2, th, ph), minlength=48)
    exp = n / 48
    assert np.all(np.abs(counts - exp) < 6 * math.sqrt(exp))
    # points are assigned to a pixel whose centre is among the closest few
    t, f = orc.pix2ang_ring(2, np.arange(48))
    cen = np.stack([np.sin(t) * np.cos(f), np.sin(t) * np.sin(f), np.cos(t)], 1)
    pts = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)[:2000]
    got = orc.ang2pix_ring(2, th[:2000], ph[:2000])
    d = pts @ cen.T
    rank = (d > d[np.arange(2000), got][:, None]).sum(1)
    assert rank.max() <= 3


def test_healpix_pixel_geometry_8192(orc):
    g = GOLD["healpix_8192"]
    area_sr = 4 * math.pi / (12 * g["nside"] ** 2)
    arcmin2 = area_sr * (180 * 60 / math.pi) ** 2
    assert abs(arcmin2 - g["area_arcmin2"]) < 5e-4
    assert abs(math.sqrt(area_sr) / ARCSEC - g["length_arcsec"]) < 0.05
    # samples at Nside 8192 round-trip, including cap/belt edges and phi wrap
    N = g["nside"]
    ncap = 2 * N * (N - 1)
    sample = np.array([0, 1, 3, 4, ncap - 1, ncap, ncap + 1, ncap + 4 * N - 1, 6 * N * N, 12 * N * N - 1,
                       12 * N * N - ncap - 1, 12 * N * N - ncap, 123456789, 805306367 - 5])
    th, ph = orc.pix2ang_ring(N, sample)
    assert np.array_equal(orc.ang2pix_ring(N, th, ph), sample)
    gf = GOLD["flat_pixel"]
    assert abs(gf["field_deg"] * 3600 / gf["n"] - gf["pixel_arcsec"]) < 5e-3


def test_hp_healpix_conservation_and_sign(orc, params):
    """The oracle's HEALPix HP map (r_perp = D_A sin psi on the sphere, Sec. 5.2 maps) for one nearby halo:
    the sum of y over the pixels times the pixel solid angle is the integral of y over the solid angle of
    the footprint, int_0^psi_t y(D_A sin psi) 2 pi sin psi dpsi, to the pixel-centre sampling error; the
    pixel nearest the centre holds the line-of-sight integral at its own r_perp; the kSZ map changes sign
    with v."""
    M, c, z, th0, ph0 = 2e14, 5.0, 0.05, 1.0, 2.0
    h = orc.solve_halo(params, M, c, z)
    assert h.status == 0
    nside = 4096
    pixsize = math.sqrt(4 * math.pi / (12 * nside * nside))
    psi_t = math.asin(h.R_t / h.D_A)
    # every pixel whose centre can lie within psi_t: a grid of directions at a third of the pixel size
    g = np.arange(-psi_t - 2 * pixsize, psi_t + 2 * pixsize, pixsize / 3)
    gt = (th0 + g[:, None] + 0 * g[None, :]).ravel()
    gp = (ph0 + g[None, :] / math.sin(th0) + 0 * g[:, None]).ravel()
    pix = np.unique(orc.ang2pix_ring(nside, gt, gp))
    pt, pp = orc.pix2ang_ring(nside, pix)
    cospsi = np.sin(pt) * math.sin(th0) * np.cos(pp - ph0) + np.cos(pt) * math.cos(th0)
    pix = pix[cospsi > math.cos(psi_t + pixsize)]
    assert len(pix) > 3000
    halos = orc.solve_halos(params, [M], [c], [z])
    cat = dict(theta=[th0], phi=[ph0], v_los=[300.0])
    y, b = orc.hp_healpix_pixels(params, halos, cat, nside, pix)
    y2, b2 = orc.hp_healpix_pixels(params, halos, dict(cat, v_los=[-300.0]), nside, pix)
    assert np.array_equal(y2, y) and np.array_equal(b2, -b)
    # no footprint pixel left out: the ring of candidates beyond psi_t is empty
    pt, pp = orc.pix2ang_ring(nside, pix)
    cospsi = np.sin(pt) * math.sin(th0) * np.cos(pp - ph0) + np.cos(pt) * math.cos(th0)
    psi = np.arccos(np.clip(cospsi, -1, 1))
    assert np.all(y[psi > psi_t * (1 + 1e-9)] == 0) and np.all(y[psi < psi_t * (1 - 1e-6)] > 0)
    ref = integrate.quad(lambda a: orc.los(params, h, h.D_A * math.sin(a))[0] * 2 * math.pi * math.sin(a), 0, psi_t,
                         points=[math.asin(h.r_vir / h.D_A)] if h.r_vir < h.R_t else None, epsabs=0,
                         epsrel=1e-10, limit=200)[0]
    Ymap = y.sum() * 4 * math.pi / (12 * nside * nside)
    assert abs(Ymap / ref - 1) < 2e-3
    k = int(np.argmin(psi))
    # sin(psi) of that pixel from the cross product of the unit vectors (arccos loses digits near 0)
    pv = np.array([math.sin(pt[k]) * math.cos(pp[k]), math.sin(pt[k]) * math.sin(pp[k]), math.cos(pt[k])])
    hv = np.array([math.sin(th0) * math.cos(ph0), math.sin(th0) * math.sin(ph0), math.cos(th0)])
    sinpsi = float(np.linalg.norm(np.cross(pv, hv)))
    assert abs(y[k] / orc.los(params, h, h.D_A * sinpsi)[0] - 1) < 1e-12


# ----------------------------------------------------------------------- PP --
def test_sph_kernel_integral(orc):
    g = GOLD["sph_kernel_norm"]
    tot = integrate.quad(lambda x: orc.W_sph(x), -1, 1, points=[-0.5, 0, 0.5], epsabs=0, epsrel=2e-14)[0]
    assert abs(tot - g["integral_of_shape"]) < 1e-14
    for x in np.linspace(-1.2, 1.2, 49):
        ref = integrate.quad(lambda t: orc.W_sph(t), -1, x, points=[p for p in (-0.5, 0, 0.5) if -1 < p < x] or None,
                             epsabs=0, epsrel=2e-14)[0] / tot if x > -1 else 0.0
        assert abs(orc.w_sph(x) - ref) < 1e-13
    for x in (-1.0, -0.5, 0.0, 0.5, 1.0):       # continuity at the branch points
        assert abs(orc.w_sph(x - 1e-12) - orc.w_sph(x + 1e-12)) < 1e-11
    assert orc.w_sph(0.0) == 0.5


def test_knn_brute_force_vs_kdtree(orc):
    rng = np.random.default_rng(3)
    X = rng.normal(size=(1500, 3)) * np.array([1.0, 2.0, 0.5])
    h = orc.knn_h(X[:, 0], X[:, 1], X[:, 2], 32)
    d, _ = cKDTree(X).query(X, k=33)
    assert np.allclose(h, d[:, 32], rtol=1e-14, atol=0)
    # the query-subset form (used on samples of large sets) against the same tree
    q = rng.choice(len(X), 40, replace=False)
    for k in (1, 7, 32, 64):
        hq = orc.knn_h_query(q, X[:, 0], X[:, 1], X[:, 2], k)
        dq, _ = cKDTree(X).query(X[q], k=k + 1)
        assert np.allclose(hq, dq[:, k], rtol=1e-14, atol=0), k


def test_pp_weights_sum_to_one_and_sign(orc, params):
    rng = np.random.default_rng(5)
    npix, pix = 64, 1e-5
    n = 300
    thx = rng.uniform(12, 52, n) * pix
    thy = rng.uniform(12, 52, n) * pix
    H = rng.uniform(0.3, 10, n) * pix
    ay = rng.uniform(0, 1, n)
    ab = rng.normal(size=n)
    y, b = orc.pp_deposit(thx, thy, H, ay, ab, npix, pix)
    assert abs(y.sum() / ay.sum() - 1) < 1e-13
    assert abs(b.sum() - ab.sum()) < 1e-12 * np.abs(ab).sum()
    y2, b2 = orc.pp_deposit(thx, thy, H, ay, -ab, npix, pix)
    assert np.array_equal(b2, -b)
    # a particle centred in a pixel with H < pix/2 deposits everything there
    y1, _ = orc.pp_deposit([10.5 * pix], [20.5 * pix], [0.4 * pix], [1.0], [0.0], npix, pix)
    assert y1[20, 10] == 1.0


def test_pp_amplitudes_definitions(orc, params):
    h = orc.solve_halo(params, 1e14, 5.0, 0.5)
    halos = (orc.Halo * 1)(h)
    pix = 5 * math.pi / 180 / 4096
    r = np.array([0.01, 0.3, h.r_f * 0.999, h.r_f * 1.2, 0.2])
    hid = np.array([0, 0, 0, 0, -1], dtype=np.int32)
    z = np.array([0.5, 0.5, 0.5, 0.5, 0.7])
    v = np.array([100.0, -50.0, 20.0, 30.0, 400.0])
    Mp = 4.7e10
    ay, ab = orc.pp_amplitudes(params, halos, z, v, hid, r, Mp, pix)
    u = orc.MPC / params.h
    Lpix = orc.D_A(params, 0.5) * u * pix
    rho_s = h.rho_s * orc.MSUN / params.h / u ** 3
    x = r[1] / h.r_s
    V = Mp * orc.MSUN / params.h / (rho_s / (x * (1 + x) ** 2))
    Pe, ne = orc.profile(params, h, r[1])
    assert abs(ay[1] / (orc.SIGMA_T / orc.ME_C2 * Pe * V / Lpix ** 2) - 1) < 1e-13
    assert abs(ab[1] / (orc.SIGMA_T * (-50e5 / orc.C_CGS) * math.exp(-orc.tau(params, 0.5)) * ne * V / Lpix ** 2) - 1) < 1e-13
    assert ay[3] == 0 and ab[3] == 0
    Lf = orc.D_A(params, 0.7) * u * pix
    fb = params.Omega_b / params.Omega_m
    ref = orc.SIGMA_T * 400e5 / orc.C_CGS * fb * Mp * orc.MSUN / params.h / (2 / (1 + params.X_H) * orc.M_P) \
        * math.exp(-orc.tau(params, 0.7)) / Lf ** 2
    assert ay[4] == 0 and abs(ab[4] / ref - 1) < 1e-13


# ---------------------------------------------------------- effective-neighbour smoothing length --
# h solves N_eff(h) = (4 pi/3) h^3 sum_j W(r_ij, h) = (32/3) sum_j W_shape(r_ij/h), self included
# (Sec. 3.4, Eq. SPH_kernel; reading: the standard SPH density sum).

def _sphere(m, d, rng):
    v = rng.normal(size=(m, 3))
    v *= d / np.linalg.norm(v, axis=1)[:, None]
    return np.vstack([np.zeros((1, 3)), v])       # the query at the origin, m points at distance d


def test_neff_sphere_closed_forms(orc):
    """m points at one distance d: N_eff = (32/3)(1 + m W(d/h)) = 64 gives W(d/h) = 5/m.  m = 10 lands
    on the inner branch (1 - 6x^2 + 6x^3 = 1/2, a cubic solved by numpy), m = 40 on the outer one
    (2 (1 - x)^3 = 1/8, x = 1 - 16^(-1/3)).  Dropping the self term, or the 32/3, moves both."""
    rng = np.random.default_rng(41)
    d = 0.37
    P = _sphere(10, d, rng)
    roots = np.roots([6.0, -6.0, 0.0, 0.5])
    x = [r.real for r in roots if abs(r.imag) < 1e-12 and 0.0 < r.real < 0.5]
    assert len(x) == 1
    h = orc.neff_h_query([0], P[:, 0], P[:, 1], P[:, 2], 64.0)[0]
    assert abs(h / (d / x[0]) - 1) < 1e-12
    P = _sphere(40, d, rng)
    h = orc.neff_h_query([0], P[:, 0], P[:, 1], P[:, 2], 64.0)[0]
    assert abs(h / (d / (1.0 - 16.0 ** (-1.0 / 3.0))) - 1) < 1e-12


def test_neff_lattice_continuum_limit(orc):
    """On a simple cubic lattice the kernel-weighted count tends to the number of points in the
    sphere, (4 pi/3)(h/a)^3 (the kernel integrates to one): within 1e-3 at N = 64, 200, 500."""
    g = np.arange(-10, 11, dtype=np.float64)
    X, Y, Z = [v.ravel() for v in np.meshgrid(g, g, g, indexing="ij")]
    i0 = int(np.nonzero((X == 0) & (Y == 0) & (Z == 0))[0][0])
    for N in (64.0, 200.0, 500.0):
        h = orc.neff_h_query([i0], X, Y, Z, N)[0]
        assert abs(h / (3 * N / (4 * np.pi)) ** (1.0 / 3.0) - 1) < 1e-3


def test_neff_scaling_and_root(orc):
    """Scaling every position by s scales h by s; at the returned h the count is n_ngb."""
    rng = np.random.default_rng(42)
    X, Y, Z = rng.random((3, 3000))
    q = [0, 17, 999]
    h = orc.neff_h_query(q, X, Y, Z, 64.0)
    hs = orc.neff_h_query(q, 3.7 * X, 3.7 * Y, 3.7 * Z, 64.0)
    assert np.all(np.abs(hs / (3.7 * h) - 1) < 1e-12)
    for i, hh in zip(q, h):
        assert abs(orc.neff_at(X, Y, Z, i, hh) - 64.0) < 1e-9


# ------------------------------------------------------ all-sky nearest-pixel kSZ (App. A) --
def _ring_centres(N):
    """RING-ordered pixel centres (z = cos theta, phi) from the closed forms of Gorski et al. (2005):
    polar rings z = 1 - i^2/(3N^2), phi = pi/(2i) (j - 1/2); belt rings z = 4/3 - 2i/(3N) with
    4N centres spaced pi/(2N), starting at phi = 0 on rings with i - N odd and half a spacing later
    on the others (so the four equatorial base pixels of N = 1 sit at phi = 0, pi/2, pi, 3pi/2 and
    the polar ones at pi/4 + k pi/2); the south cap mirrors the north."""
    zs, phis = [], []
    for i in range(1, 4 * N):
        if i < N or i > 3 * N:
            k = i if i < N else 4 * N - i
            z = 1 - k * k / (3.0 * N * N)
            z = z if i < N else -z
            j = np.arange(1, 4 * k + 1)
            phi = math.pi / (2 * k) * (j - 0.5)
        else:
            z = 4.0 / 3 - 2.0 * i / (3 * N)
            j = np.arange(1, 4 * N + 1)
            phi = math.pi / (2 * N) * (j - (1.0 if (i - N) % 2 else 0.5))
        zs.append(np.full(len(j), z))
        phis.append(phi)
    return np.concatenate(zs), np.concatenate(phis)


def _unit(z, phi):
    s = np.sqrt(np.maximum(0.0, 1 - z * z))
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


@pytest.mark.parametrize("N", [1, 4, 8])
def test_ngp_pixel_is_nearest_centre(orc, params, N):
    # directions within a tenth of a pixel of a pixel centre land in that pixel, which is also the
    # pixel with the nearest centre found by brute force over all 12 N^2 centres
    zc, phic = _ring_centres(N)
    assert len(zc) == 12 * N * N
    rng = np.random.default_rng(11)
    pick = rng.integers(0, len(zc), 600)
    c = _unit(zc[pick], phic[pick])
    t = rng.normal(size=c.shape)
    t -= (t * c).sum(1)[:, None] * c
    t /= np.linalg.norm(t, axis=1)[:, None]
    d = 0.1 * math.sqrt(4 * math.pi / (12 * N * N)) * rng.random(len(pick))[:, None]
    u = c * np.cos(d) + t * np.sin(d)
    theta = np.arccos(np.clip(u[:, 2], -1, 1))
    phi = np.arctan2(u[:, 1], u[:, 0])
    pix, _ = orc.pp_healpix_ngp(params, theta, phi, np.full(len(pick), 0.5), np.full(len(pick), 100.0), 1e10, N)
    nearest = np.argmax(u @ _unit(zc, phic).T, axis=1)
    assert np.array_equal(pix, pick)
    assert np.array_equal(pix, nearest)


def test_ngp_amplitude_and_map_invariants(orc, params):
    # b_i = sigma_T (v/c) (f_gas M_p/(mu_e m_p)) e^-tau / (D_A^2 Omega_pix), Omega_pix = 4 pi/(12 N^2)
    # (Eq. field_b with the HEALPix pixel area); the whole amplitude in one pixel
    N, Mp = 16, 3.1e10
    rng = np.random.default_rng(5)
    n = 400
    theta = np.arccos(rng.uniform(-1, 1, n))
    phi = rng.uniform(-4, 10, n)
    z = rng.uniform(0.01, 3.7, n)
    v = rng.normal(0, 300, n)
    theta[:3] = [0.0, math.pi, -0.1]                  # both poles are valid; a negative colatitude is not
    pix, amp = orc.pp_healpix_ngp(params, theta, phi, z, v, Mp, N)
    u = orc.MPC / params.h
    fb = params.Omega_b / params.Omega_m
    omega = math.pi / (3 * N * N)
    for i in (0, 1, 7, 100):
        ref = orc.SIGMA_T * v[i] * 1e5 / orc.C_CGS * fb * Mp * orc.MSUN / params.h \
            / (2 / (1 + params.X_H) * orc.M_P) * math.exp(-orc.tau(params, z[i])) / ((orc.D_A(params, z[i]) * u) ** 2 * omega)
        assert abs(amp[i] / ref - 1) < 1e-13
    assert pix[0] < 4 and 12 * N * N - 4 <= pix[1] < 12 * N * N       # first and last ring hold 4 pixels
    assert pix[2] == -1 and amp[2] == 0
    b, babs = orc.pp_healpix_ngp_map(params, theta, phi, z, v, Mp, N)
    assert abs(b.sum() - amp.sum()) < 1e-12 * np.abs(amp).sum()
    assert abs(babs.sum() - np.abs(amp).sum()) < 1e-12 * np.abs(amp).sum()
    b2, _ = orc.pp_healpix_ngp_map(params, theta, phi, z, -v, Mp, N)
    assert np.array_equal(b2, -b)
    # the map is additive over particle subsets
    bA, _ = orc.pp_healpix_ngp_map(params, theta[:150], phi[:150], z[:150], v[:150], Mp, N)
    bB, _ = orc.pp_healpix_ngp_map(params, theta[150:], phi[150:], z[150:], v[150:], Mp, N)
    assert np.allclose(bA + bB, b, rtol=0, atol=1e-13 * np.abs(amp).max())


def test_field_tsz_amplitude(orc, params):
    # filament extension of Eq. field_y: P_e = n_e k_B T, so y_i / b_i = (k_B T / m_e c^2) / ((v/c) e^-tau)
    # for the same particle (same electron count and pixel area); T = 0 is the paper's y = 0
    import copy
    p = copy.copy(params)
    z, v = np.array([0.3, 1.1]), np.array([250.0, -80.0])
    hid = np.array([-1, -1], dtype=np.int32)
    pix = 1e-4
    ay0, ab0 = orc.pp_amplitudes(p, None, z, v, hid, np.zeros(2), 2e9, pix)
    assert np.all(ay0 == 0)
    p.field_T = 1e4
    ay, ab = orc.pp_amplitudes(p, None, z, v, hid, np.zeros(2), 2e9, pix)
    kB, mec2, c = 1.380649e-16, 8.1871057769e-7, 2.99792458e10
    for i in range(2):
        ratio = (kB * 1e4 / mec2) / (v[i] * 1e5 / c * math.exp(-orc.tau(p, z[i])))
        assert abs(ay[i] / ab[i] / ratio - 1) < 1e-13
    assert np.array_equal(ab, ab0)
    p.field_T = 3e4
    ay3, _ = orc.pp_amplitudes(p, None, z, v, hid, np.zeros(2), 2e9, pix)
    assert np.allclose(ay3, 3 * ay, rtol=1e-14, atol=0)


# ------------------------------------------------- flat-sky power spectrum (Sec. 5.3) --
def test_spectrum_parseval_and_cosine():
    from oracle import spectrum as S
    rng = np.random.default_rng(3)
    n, d = 64, 2e-4
    f = rng.normal(size=(n, n))
    lb, cl, cnt = S.flat_power_spectrum(f, d, np.array([0.0, 1e12]))
    assert cnt[0] == n * n
    assert abs(cl[0] * cnt[0] / (d * d * (f * f).sum()) - 1) < 1e-12        # Parseval
    # one cosine of wave vector (a, b): power d^2 N^2 / 4 on each of the modes +-(a, b), nothing else
    a, b = 5, 3
    x = np.arange(n)
    g = np.cos(2 * math.pi * (a * x[None, :] + b * x[:, None]) / n)
    L = n * d
    l0 = 2 * math.pi / L * math.hypot(a, b)
    lb, cl, cnt = S.flat_power_spectrum(g, d, np.array([0.999 * l0, 1.001 * l0]))
    same = sum(1 for i in range(-n // 2, n // 2) for j in range(-n // 2, n // 2) if i * i + j * j == a * a + b * b)
    assert cnt[0] == same
    assert abs(cl[0] * cnt[0] / (2 * d * d * n * n / 4) - 1) < 1e-12
    assert abs(lb[0] / l0 - 1) < 1e-14


def test_spectrum_white_noise_and_mode_counts():
    from oracle import spectrum as S
    rng = np.random.default_rng(4)
    n, d, sig = 256, 1e-4, 2.5
    f = rng.normal(0, sig, size=(n, n))
    edges = S.log_edges(30, 1e2, 1e5)
    lb, cl, cnt = S.flat_power_spectrum(f, d, edges)
    # white noise: every mode has expected power d^2 sigma^2
    big = cnt >= 1000
    assert big.sum() >= 5
    assert np.all(np.abs(cl[big] / (d * d * sig * sig) - 1) < 5 / np.sqrt(cnt[big]))
    # annuli inside the Nyquist square hold about pi (|k|^2 range) modes (Gauss circle problem)
    t = S.thresholds(edges, n, d)
    inside = np.sqrt(t[1:]) < n / 2
    expect = math.pi * (t[1:] - t[:-1])
    ok = inside & (expect > 50)
    assert ok.sum() >= 5
    assert np.all(np.abs(cnt[ok] - expect[ok]) < 4 * np.sqrt(t[1:][ok]) + 4)
    assert np.all((lb[cnt > 0] >= edges[:-1][cnt > 0]) & (lb[cnt > 0] < edges[1:][cnt > 0]))


def test_parallel_solve_equals_serial(orc, params):
    # the process pool used by the full-size parity tests returns exactly the serial solutions
    rng = np.random.default_rng(5)
    M = 10 ** rng.uniform(12.5, 15.5, 300)
    c = rng.uniform(2, 15, 300)
    z = rng.uniform(0.05, 3, 300)
    a = orc.solve_halos(params, M, c, z)
    b = orc.solve_halos_parallel(params, M, c, z, workers=4)
    for f in ("x_f", "rho0", "P0", "R_t", "D_A", "tau", "status"):
        assert [getattr(h, f) for h in a] == [getattr(h, f) for h in b], f
