"""Pins of the oracle's ICM solution and sight-line projection that do not go through the oracle's
own residual functions.

- The gas of a solved halo is recomputed here from its printed definitions (Sec. 2.1-2.2): the NFW
  potential of the halo truncated at r_vir written out from Poisson's equation, the polytropic
  relation P_tot ~ rho_g^Gamma, the untruncated Jeans dispersion from its integral definition.
  From these the test checks hydrostatic equilibrium, the surface-pressure closure
  P_tot(r_f) = P_s (Eq. surface_pressure) and the energy balance (Eq. energy_conservation with the
  final gas energy integral and the expansion work) with scipy quadrature.
- The sight-line integral of Sec. 3.3 is checked on profiles with closed-form projections: a uniform
  sphere, the isothermal (beta = 2/3) and beta = 1 beta models, a general beta model through the
  incomplete beta function, and a profile with a jump.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

CORNERS = [(10 ** 12.5, 2.0, 0.05), (10 ** 12.5, 15.0, 3.0), (10 ** 15.5, 2.0, 3.0), (10 ** 15.5, 15.0, 0.05),
           (1e14, 5.0, 0.5), (1e13, 6.0, 2.0)]


class Gas:
    """A solved halo's structure and gas in CGS, from the definitions of Sec. 2.1-2.2."""

    def __init__(self, orc, p, h):
        self.orc, self.p, self.h = orc, p, h
        self.u = orc.MPC / p.h                      # cm per Mpc/h
        self.um = orc.MSUN / p.h                    # g per Msun/h
        self.c = h.c
        self.Mvir = h.M * self.um
        self.rv, self.rs, self.rf = h.r_vir * self.u, h.r_s * self.u, h.r_f * self.u
        self.mc = math.log1p(self.c) - self.c / (1 + self.c)
        self.rho_s = self.Mvir / (4 * math.pi * self.rs ** 3 * self.mc)
        self.G = orc.G_CGS
        self.fb = p.Omega_b / p.Omega_m
        X = p.X_H
        self.mu_e = 2 / (1 + X)
        self.pe_frac = (2 * X + 2) / (5 * X + 3)

    # --- dark matter (NFW, Sec. 2.1) ---
    def rho(self, r):
        x = r / self.rs
        return self.rho_s / (x * (1 + x) ** 2)

    def M_enc(self, r):
        """Untruncated NFW enclosed mass (the halo holds M_vir inside r_vir)."""
        x = r / self.rs
        return 4 * math.pi * self.rho_s * self.rs ** 3 * (math.log1p(x) - x / (1 + x))

    def Phi(self, r):
        """Potential of the halo truncated at r_vir: -G M(r)/r - 4 pi G int_r^rvir rho r' dr' inside,
        a point mass outside (from Poisson's equation; the integral is elementary)."""
        if r >= self.rv:
            return -self.G * self.Mvir / r
        x = r / self.rs
        shell = 4 * math.pi * self.G * self.rho_s * self.rs ** 2 * (1 / (1 + x) - 1 / (1 + self.c))
        return -self.G * self.M_enc(r) / r - shell

    def sigma2(self, r):
        """Isotropic Jeans dispersion of the untruncated halo: rho sigma^2 = int_r^inf rho G M / r'^2 dr'."""
        f = lambda t: self.rho(t) * self.G * self.M_enc(t) / t ** 2
        # in s = ln(t / r) the integrand falls like s e^(-4 s); beyond s = 40 it is below 1e-60 of its peak
        fs = lambda s: f(r * math.exp(s)) * r * math.exp(s)
        s = sum(integrate.quad(fs, a, b, epsabs=0, epsrel=1e-13, limit=200)[0] for a, b in ((0, 2), (2, 8), (8, 40)))
        return s / self.rho(r)

    # --- gas of the solved halo, from the oracle's profile of n_e ---
    def rho_g(self, r):
        return self.orc.profile(self.p, self.h, r / self.u)[1] * self.mu_e * self.orc.M_P

    def P_tot(self, r):
        """Polytropic relation P_tot = P0 (rho_g / rho0)^Gamma (Sec. 2.1)."""
        return self.h.P0 * (self.rho_g(r) / self.h.rho0) ** self.p.Gamma

    def pieces(self, lo, hi):
        """[lo, hi] split at r_vir (where the potential's second derivative jumps)."""
        if lo < self.rv < hi:
            return [(lo, self.rv), (self.rv, hi)]
        return [(lo, hi)]

    def integral(self, f, lo, hi):
        return sum(integrate.quad(f, a, b, epsabs=0, epsrel=1e-12, limit=400)[0] for a, b in self.pieces(lo, hi))


@pytest.mark.parametrize("M,c,z", CORNERS)
def test_gas_in_hydrostatic_equilibrium(orc, params, M, c, z):
    # the polytrope sits in the halo's potential: dP_tot/dr = -rho_g G M(<r) / r^2 at every r < r_f
    g = Gas(orc, params, orc.solve_halo(params, M, c, z))
    for frac in (0.05, 0.3, 0.7, 0.95):
        r = frac * g.rf
        if abs(r / g.rv - 1) < 1e-3:
            continue
        d = 1e-4 * r
        dP = (g.P_tot(r + d) - g.P_tot(r - d)) / (2 * d)
        m_in = g.M_enc(min(r, g.rv))           # the truncated halo: all of M_vir inside r_vir
        rhs = -g.rho_g(r) * g.G * m_in / r ** 2
        assert abs(dP / rhs - 1) < 1e-6, (frac, dP, rhs)


@pytest.mark.parametrize("M,c,z", CORNERS)
def test_electron_pressure_is_the_thermal_share(orc, params, M, c, z):
    # P_e = (2X+2)/(5X+3) P_tot max(0, 1 - R_nt), R_nt = alpha_nt f(z) (r/r500)^n_nt (Sec. 2.3, 3.2)
    h = orc.solve_halo(params, M, c, z)
    g = Gas(orc, params, h)
    fz = min((1 + z) ** params.beta_nt, (4 ** -params.n_nt / params.alpha_nt - 1) * math.tanh(params.beta_nt * z) + 1)
    for frac in (0.1, 0.5, 0.9, 0.99):
        r = frac * g.rf
        Rnt = params.alpha_nt * fz * (r / (h.r500 * g.u)) ** params.n_nt
        Pe = orc.profile(params, h, r / g.u)[0]
        want = g.pe_frac * g.P_tot(r) * max(0.0, 1 - Rnt)
        assert abs(Pe - want) <= 1e-12 * g.pe_frac * g.P_tot(r), (frac, Pe, want)


@pytest.mark.parametrize("M,c,z", CORNERS)
def test_surface_pressure_closure(orc, params, M, c, z):
    # Eq. surface_pressure: the total gas pressure just inside r_f equals P_s = f_b rho_NFW(r_vir) sigma^2(r_vir),
    # with sigma^2 from the Jeans integral of the untruncated halo (reading R4)
    h = orc.solve_halo(params, M, c, z)
    g = Gas(orc, params, h)
    Ps = g.fb * g.rho(g.rv) * g.sigma2(g.rv)
    assert abs(Ps / h.P_s - 1) < 1e-10
    assert abs(g.P_tot(g.rf * (1 - 1e-13)) / Ps - 1) < 1e-9


@pytest.mark.parametrize("M,c,z", CORNERS)
def test_energy_balance_from_definitions(orc, params, M, c, z):
    # Eq. energy_conservation (reading R2: injected energy and expansion work raise the gas energy):
    #   E_gf = E_gi + eps_DM |E_DM| + eps_* M_* c^2 + dE_p
    # E_gf = int_0^rf 4 pi r^2 [3/2 P_tot + rho_g Phi] dr (the final gas energy, P_tot not P_th);
    # E_gi = f_b int_r*^rvir 4 pi r^2 rho [3/2 sigma^2 + Phi] dr (the initial energy, no 1/2 on Phi, R3);
    # dE_p = (4 pi / 3)(r_vir^3 - r_f^3) P_s.
    h = orc.solve_halo(params, M, c, z)
    assert h.status == 0
    g = Gas(orc, params, h)
    Egf = g.integral(lambda r: 4 * math.pi * r * r * (1.5 * g.P_tot(r) + g.rho_g(r) * g.Phi(r)), 0.0, g.rf)
    rstar = h.x_star * g.rs
    Egi = g.fb * integrate.quad(lambda r: 4 * math.pi * r * r * g.rho(r) * (1.5 * g.sigma2(r) + g.Phi(r)),
                                rstar, g.rv, epsabs=0, epsrel=1e-11, limit=200)[0]
    assert abs(Egi / h.E_gi - 1) < 1e-9
    Ps = g.fb * g.rho(g.rv) * g.sigma2(g.rv)
    dEp = 4 * math.pi / 3 * (g.rv ** 3 - g.rf ** 3) * Ps
    inj = params.eps_star * h.M_star * g.um * orc.C_CGS ** 2      # eps_DM = 0 (Table 1)
    assert params.eps_DM == 0.0
    assert abs(Egf - (Egi + inj + dEp)) < 1e-8 * abs(Egi), (Egf, Egi, inj, dEp)
    # every term matters at this tolerance: a dropped term or a flipped sign fails
    for wrong in (Egi + dEp, Egi + inj - dEp, Egi - inj + dEp):
        assert abs(Egf - wrong) > 1e-6 * abs(Egi)
    # P_th in place of P_tot in the final energy also fails where the non-thermal share is non-zero
    Egf_th = g.integral(lambda r: 4 * math.pi * r * r * (1.5 * orc.profile(params, h, r / g.u)[0] / g.pe_frac
                                                         + g.rho_g(r) * g.Phi(r)), 0.0, g.rf)
    assert abs(Egf_th - (Egi + inj + dEp)) > 1e-6 * abs(Egi)


def test_potential_matches_poisson_quadrature(orc, params):
    # the closed-form potential used above against -G M(r)/r - 4 pi G int_r^rvir rho r' dr' by quadrature
    g = Gas(orc, params, orc.solve_halo(params, 1e14, 5.0, 0.5))
    for frac in (0.01, 0.3, 0.99):
        r = frac * g.rv
        q = -g.G * g.M_enc(r) / r - 4 * math.pi * g.G * integrate.quad(lambda t: g.rho(t) * t, r, g.rv, epsabs=0,
                                                                      epsrel=1e-13)[0]
        assert abs(g.Phi(r) / q - 1) < 1e-12
    assert abs(g.Phi(g.rv * (1 - 1e-12)) / g.Phi(g.rv) - 1) < 1e-10     # continuous at r_vir


# ----------------------------------------------------- sight-line projection (Sec. 3.3) --
@pytest.mark.parametrize("frac", [0.0, 0.3, 0.9, 0.999])
def test_los_uniform_sphere(orc, frac):
    rmax = 2.5
    R = frac * rmax
    assert abs(orc.los_model(0, 0, 0, rmax, R) / (2 * math.sqrt(rmax ** 2 - R ** 2)) - 1) < 1e-12
    assert orc.los_model(0, 0, 0, rmax, rmax) == 0.0 and orc.los_model(0, 0, 0, rmax, 1.1 * rmax) == 0.0


@pytest.mark.parametrize("R", [0.0, 0.05, 0.4, 1.7, 2.9])
def test_los_isothermal_beta_model(orc, R):
    # beta = 2/3: f = 1 / (1 + r^2/rc^2); through a sphere of radius rmax the projection is
    # 2 rc^2 atan(L / a) / a with a^2 = rc^2 + R^2, L^2 = rmax^2 - R^2
    rc, rmax = 0.3, 3.0
    a, L = math.hypot(rc, R), math.sqrt(rmax ** 2 - R ** 2)
    want = 2 * rc ** 2 * math.atan(L / a) / a
    assert abs(orc.los_model(1, 2.0 / 3.0, rc, rmax, R) / want - 1) < 1e-11


@pytest.mark.parametrize("R", [0.0, 0.2, 1.0, 2.5])
def test_los_beta_one(orc, R):
    # beta = 1: f = (1 + r^2/rc^2)^(-3/2); projection 2 rc^3 L / (a^2 sqrt(rc^2 + rmax^2))
    rc, rmax = 0.5, 3.0
    a2, L = rc ** 2 + R ** 2, math.sqrt(rmax ** 2 - R ** 2)
    want = 2 * rc ** 3 * L / (a2 * math.sqrt(rc ** 2 + rmax ** 2))
    assert abs(orc.los_model(1, 1.0, rc, rmax, R) / want - 1) < 1e-11


@pytest.mark.parametrize("beta", [0.55, 0.8, 1.3])
def test_los_general_beta_model(orc, beta):
    # f = rc^(2p) (a^2 + l^2)^(-p), p = 3 beta / 2: int_0^L (a^2 + l^2)^(-p) dl = a^(1-2p) B(u; 1/2, p - 1/2) / 2,
    # u = L^2 / (a^2 + L^2), B the (unregularised) incomplete beta function (scipy's betainc x beta);
    # as rmax -> inf this tends to the textbook sqrt(pi) rc Gamma(p - 1/2)/Gamma(p) (1 + R^2/rc^2)^(1/2 - p)
    rc, p = 0.4, 1.5 * beta
    for R, rmax in ((0.0, 3.0), (0.7, 3.0), (1.5, 2.0)):
        a2, L2 = rc ** 2 + R ** 2, rmax ** 2 - R ** 2
        u = L2 / (a2 + L2)
        want = rc ** (2 * p) * a2 ** (0.5 - p) * special.betainc(0.5, p - 0.5, u) * special.beta(0.5, p - 0.5)
        assert abs(orc.los_model(1, beta, rc, rmax, R) / want - 1) < 1e-10, (R, rmax)
    if beta > 1.0:
        R, rmax = 0.3, 1e4
        inf = math.sqrt(math.pi) * rc * special.gamma(p - 0.5) / special.gamma(p) * (1 + R * R / rc / rc) ** (0.5 - p)
        assert abs(orc.los_model(1, beta, rc, rmax, R) / inf - 1) < 1e-6


@pytest.mark.parametrize("R", [0.0, 0.6, 0.999, 1.0, 1.4])
def test_los_profile_with_a_jump(orc, R):
    # f = 1 inside r1, f2 between r1 and rmax: 2 [f2 sqrt(rmax^2 - R^2) + (1 - f2) sqrt(r1^2 - R^2)] inside r1
    r1, f2, rmax = 1.0, 0.25, 2.0
    want = 2 * f2 * math.sqrt(rmax ** 2 - R ** 2)
    if R < r1:
        want += 2 * (1 - f2) * math.sqrt(r1 ** 2 - R ** 2)
    assert abs(orc.los_model(2, r1, f2, rmax, R) / want - 1) < 1e-12


# ------------------------------------------------------------ cross-method (Sec. 3.3 vs Sec. 3.4) --
def test_pp_of_a_sampled_halo_converges_to_hp(orc):
    """Particle-based pasting of a spherical NFW halo sampled with 1e6 particles against halo-based
    pasting of the same solved halo.  Each particle carries P_e(r_i) M_p / rho_NFW(r_i) (Sec. 3.4), an
    unbiased Monte Carlo estimate of the gas integral that the HP projection (Sec. 3.3) integrates
    exactly; each particle footprint's weights sum to one, so the PP map total is the sum of the
    amplitudes.  The footprint cut is moved past r_f so both methods see all of the gas."""
    p = orc.default_params(trunc_r500=1e3)
    h = orc.solve_halo(p, 1e14, 5.0, 0.3)
    assert h.status == 0 and h.R_t == h.r_f
    rng = np.random.default_rng(7)
    n = 1_000_000
    m = lambda x: np.log1p(x) - x / (1 + x)
    xmax = h.r_f / h.r_s
    target = rng.uniform(size=n) * m(xmax)          # radii from the NFW enclosed-mass CDF inside r_f
    lo, hi = np.zeros(n), np.full(n, xmax)
    for _ in range(64):
        mid = 0.5 * (lo + hi)
        above = m(mid) > target
        hi, lo = np.where(above, mid, hi), np.where(above, lo, mid)
    r = 0.5 * (lo + hi) * h.r_s
    M_p = h.M * m(xmax) / m(h.c) / n                # untruncated NFW mass inside r_f, shared out
    pix = 2 * h.R_t / h.D_A / 300                    # footprint radius 150 pixels
    ay, ab = orc.pp_amplitudes(p, (orc.Halo * 1)(h), np.full(n, h.z), np.full(n, 300.0), np.zeros(n, np.int32), r,
                               M_p, pix)
    npix = 320
    cat = dict(theta_x=np.array([npix / 2 * pix]), theta_y=np.array([npix / 2 * pix]), v_los=np.array([300.0]))
    y, b = orc.hp_flat_solved(p, (orc.Halo * 1)(h), cat, npix, pix)
    for amp, hp in ((ay, y.sum()), (ab, b.sum())):
        sigma = amp.std() / math.sqrt(n) / amp.mean()
        err = amp.sum() / hp - 1
        # Monte Carlo error (about 2e-4 here) plus the pixel-centre sum of the HP map (about 1e-4)
        assert abs(err) < 4 * sigma + 2e-4, (err, sigma)
        assert sigma < 5e-4
