/*
 * bp_oracle.c -- FP64 CPU oracle of the baryon-pasting method
 * (Osato & Nagai 2022, "Baryon Pasting Algorithm: Halo-based and
 * Particle-based Pasting Methods", MNRAS).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, single-threaded
 * reference that the HIP library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it; the
 * product path never links, imports or calls it, and it shares no code,
 * header, table or constant with the HIP library.
 *
 * Everything is double precision and follows the paper's definitions in the
 * paper's order.  Integrals use adaptive Gauss-Kronrod (7/15) quadrature,
 * roots use Brent's method on a bracket.  Closed forms that exist only as
 * cross-checks (Lokas & Mamon velocity dispersion, energies by parts) are
 * exported separately so the tests can pin one against the other.
 *
 * Readings where the paper is silent or garbled are flagged "reading:" in
 * the comments; each one is listed in the design notes.
 *
 * Parity status of the composite ICM amplitude: the paper prints no worked
 * halo solution, so the solved (rho0, P0, r_f) are pinned only through their
 * pieces (closed forms, boundary-condition residuals), not against a printed
 * value.
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Physical constants (CGS).  CODATA-2018 and IAU nominal values; the paper  */
/* prints none of them (reading).                                            */
/* ------------------------------------------------------------------------ */
#define ORC_SIGMA_T   6.6524587321e-25      /* Thomson cross-section [cm^2] */
#define ORC_ME_C2     8.1871057769e-7       /* electron rest energy [erg]   */
#define ORC_C         2.99792458e10         /* speed of light [cm/s]        */
#define ORC_MP        1.67262192369e-24     /* proton mass [g]              */
#define ORC_G         6.67430e-8            /* Newton constant [cgs]        */
#define ORC_MSUN      1.988409870698051e33  /* solar mass [g]               */
#define ORC_MPC       3.0856775814913673e24 /* megaparsec [cm]              */
#define ORC_PI        3.14159265358979323846
#define ORC_KB        1.380649e-16          /* Boltzmann constant [erg/K]   */

/* status codes (bit flags, 0 = converged) */
#define ORC_OK            0
#define ORC_NO_BRACKET    1   /* energy residual has no sign change on the scan */
#define ORC_MULTI_ROOT    2   /* more than one sign change: first one taken     */
#define ORC_NO_STAR_ROOT  4   /* stellar mass >= baryon mass: r_* undefined     */
#define ORC_NONFINITE     8
#define ORC_BAD_INPUT     16

/* Model parameters.  Layout mirrored by the Python ctypes shim. */
typedef struct {
    double Omega_m, Omega_b, h;             /* flat LCDM, no radiation (Sec. 1) */
    double Gamma, eps_DM, eps_star, f_star, S_star;   /* Table 1 */
    double alpha_nt, beta_nt, n_nt;         /* Table 1 */
    double X_H;                             /* hydrogen mass fraction (Sec. 3.2) */
    double trunc_r500;                      /* projected footprint cut, units of r500 */
    double field_gas_frac;                  /* gas fraction of a field particle */
    double field_T;                         /* field gas temperature [K] for its tSZ (0: none) */
    int    energy_sign;                     /* 0: feedback adds gas energy; 1: as printed */
    int    pad_;
} orc_params;

/* Per-halo solution.  Halo-structure lengths are physical Mpc/h, masses
 * Msun/h; gas quantities are CGS. */
typedef struct {
    double M, c, z;
    double E, rho_crit, Delta_vir;          /* rho_crit in (Msun/h)/(Mpc/h)^3 */
    double r_vir, r_s, rho_s;
    double x500, r500, M500;
    double F_star, M_star, x_star;
    double sigma2_vir;                      /* [cm^2/s^2] */
    double P_s;                             /* [erg/cm^3] */
    double E_gi, E_DM;                      /* [erg] */
    double a, x_f, r_f;                     /* polytrope slope parameter, r_f/r_vir, r_f [Mpc/h] */
    double rho0, P0;                        /* [g/cm^3], [erg/cm^3] */
    double res_M, res_P, res_E;             /* relative residuals of the 3 conditions */
    double chi, D_A, tau;                   /* comoving Mpc/h, physical Mpc/h, optical depth */
    double f_nt, r_nt;                      /* f(z); radius where R_nt = 1 [Mpc/h] */
    double R_t;                             /* footprint radius min(r_f, trunc*r500) [Mpc/h] */
    int    status, n_sign_changes;
} orc_halo;

/* ======================================================================== */
/* Adaptive Gauss-Kronrod quadrature (7-point Gauss / 15-point Kronrod).     */
/* ======================================================================== */
typedef double (*orc_fn)(double x, void *ctx);

static const double GK_X[8] = {
    0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
    0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
    0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
    0.207784955007898467600689403773245, 0.0};
static const double GK_WK[8] = {
    0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
    0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
    0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
    0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
static const double GK_WG[4] = {
    0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
    0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

static void gk15(orc_fn f, void *ctx, double a, double b, double *res, double *err)
{
    double mid = 0.5 * (a + b), half = 0.5 * (b - a);
    double fc = f(mid, ctx);
    double rk = fc * GK_WK[7], rg = fc * GK_WG[3];
    for (int j = 0; j < 7; j++) {
        double dx = half * GK_X[j];
        double s = f(mid - dx, ctx) + f(mid + dx, ctx);
        rk += GK_WK[j] * s;
        if (j & 1) rg += GK_WG[j / 2] * s;
    }
    *res = rk * half;
    *err = fabs((rk - rg) * half);
}

/* Globally adaptive: repeatedly bisect the sub-interval with the largest
 * error estimate until the summed estimate meets the tolerance or the
 * interval budget is spent (the K15 - G7 difference overestimates the K15
 * error by orders of magnitude, so the budget is rarely reached). */
#define QUAD_MAXSEG 400
static double quad(orc_fn f, void *ctx, double a, double b, double rel_tol, double abs_tol)
{
    if (b == a) return 0.0;
    double lo[QUAD_MAXSEG], hi[QUAD_MAXSEG], rs[QUAD_MAXSEG], es[QUAD_MAXSEG];
    int n = 1;
    lo[0] = a; hi[0] = b;
    gk15(f, ctx, a, b, &rs[0], &es[0]);
    for (;;) {
        double tot = 0.0, err = 0.0;
        int worst = 0;
        for (int k = 0; k < n; k++) {
            tot += rs[k]; err += es[k];
            if (es[k] > es[worst]) worst = k;
        }
        double tol = fmax(abs_tol, rel_tol * fabs(tot));
        if (err <= tol || n >= QUAD_MAXSEG) return tot;
        double m = 0.5 * (lo[worst] + hi[worst]);
        if (!(m > lo[worst] && m < hi[worst])) return tot;   /* interval at machine resolution */
        lo[n] = m; hi[n] = hi[worst]; hi[worst] = m;
        gk15(f, ctx, lo[worst], hi[worst], &rs[worst], &es[worst]);
        gk15(f, ctx, lo[n], hi[n], &rs[n], &es[n]);
        n++;
    }
}

/* ======================================================================== */
/* Brent's root finder on a bracket [a,b] with f(a)*f(b) <= 0.               */
/* ======================================================================== */
static double brent(orc_fn f, void *ctx, double a, double b, double fa, double fb,
                    double xtol, int maxit)
{
    if (fa == 0.0) return a;
    if (fb == 0.0) return b;
    double c = a, fc = fa, d = b - a, e = d;
    for (int it = 0; it < maxit; it++) {
        if ((fb > 0 && fc > 0) || (fb < 0 && fc < 0)) { c = a; fc = fa; d = b - a; e = d; }
        if (fabs(fc) < fabs(fb)) { a = b; b = c; c = a; fa = fb; fb = fc; fc = fa; }
        double tol = 2.0 * 2.220446049250313e-16 * fabs(b) + 0.5 * xtol;
        double m = 0.5 * (c - b);
        if (fabs(m) <= tol || fb == 0.0) return b;
        if (fabs(e) >= tol && fabs(fa) > fabs(fb)) {
            double s = fb / fa, p, q;
            if (a == c) {            /* secant */
                p = 2.0 * m * s; q = 1.0 - s;
            } else {                 /* inverse quadratic interpolation */
                double qq = fa / fc, r = fb / fc;
                p = s * (2.0 * m * qq * (qq - r) - (b - a) * (r - 1.0));
                q = (qq - 1.0) * (r - 1.0) * (s - 1.0);
            }
            if (p > 0) q = -q; else p = -p;
            if (2.0 * p < fmin(3.0 * m * q - fabs(tol * q), fabs(e * q))) { e = d; d = p / q; }
            else { d = m; e = m; }
        } else { d = m; e = m; }
        a = b; fa = fb;
        b += (fabs(d) > tol) ? d : (m > 0 ? tol : -tol);
        fb = f(b, ctx);
    }
    return b;
}

/* ======================================================================== */
/* Cosmology: flat LCDM without radiation (Sec. 1; Sec. 3.2 for tau).        */
/* ======================================================================== */
static double hubble_E(const orc_params *p, double z)
{
    double a3 = (1.0 + z) * (1.0 + z) * (1.0 + z);
    return sqrt(p->Omega_m * a3 + 1.0 - p->Omega_m);
}

/* critical density today in (Msun/h)/(Mpc/h)^3 = 3 H0^2 / (8 pi G) with
 * H0 = 100 km/s/Mpc (the h^2 is absorbed by the h-units). */
static double rho_crit0_hunits(void)
{
    double H100 = 100.0 * 1e5 / ORC_MPC;                   /* [1/s] */
    double rho = 3.0 * H100 * H100 / (8.0 * ORC_PI * ORC_G); /* [h^2 g/cm^3] */
    return rho * ORC_MPC * ORC_MPC * ORC_MPC / ORC_MSUN;
}

struct cosmo_ctx { const orc_params *p; int kind; };

static double cosmo_integrand(double z, void *vctx)
{
    struct cosmo_ctx *cx = (struct cosmo_ctx *)vctx;
    double E = hubble_E(cx->p, z);
    if (cx->kind == 0) return 1.0 / E;                       /* comoving distance */
    return (1.0 + z) * (1.0 + z) / E;                         /* optical depth     */
}

/* comoving distance chi(z) = c int dz/H  [Mpc/h] */
double orc_chi(const orc_params *p, double z)
{
    struct cosmo_ctx cx = {p, 0};
    double c_over_H100 = ORC_C / 1e5 / 100.0;                /* c/H0 in Mpc/h */
    return c_over_H100 * quad(cosmo_integrand, &cx, 0.0, z, 1e-13, 0.0);
}

/* angular-diameter distance D_A = chi/(1+z) [physical Mpc/h] (flat universe) */
double orc_DA(const orc_params *p, double z) { return orc_chi(p, z) / (1.0 + z); }

/* mean Thomson optical depth to redshift z (Sec. 3.2):
 * tau = sigma_T nbar_e c int (1+z)^2/H dz, nbar_e = Omega_b rho_cr0/(mu_e m_p),
 * fully ionised at all z (reading). */
double orc_tau(const orc_params *p, double z)
{
    struct cosmo_ctx cx = {p, 1};
    double H0 = 100.0 * p->h * 1e5 / ORC_MPC;                /* [1/s] */
    double rho_cr0 = 3.0 * H0 * H0 / (8.0 * ORC_PI * ORC_G); /* [g/cm^3] */
    double mu_e = 2.0 / (1.0 + p->X_H);
    double ne = p->Omega_b * rho_cr0 / (mu_e * ORC_MP);
    return ORC_SIGMA_T * ne * (ORC_C / H0) * quad(cosmo_integrand, &cx, 0.0, z, 1e-13, 0.0);
}

/* ======================================================================== */
/* NFW halo (Sec. 2.1).                                                      */
/* ======================================================================== */
/* m(x) = ln(1+x) - x/(1+x), the enclosed-mass shape of an NFW profile */
double orc_m(double x)
{
    if (x < 1e-4) {   /* alternating series sum_{k>=2} (-1)^k (k-1)/k x^k */
        double s = 0.0, xk = x * x;
        for (int k = 2; k < 12; k++) { s += ((k & 1) ? -1.0 : 1.0) * (k - 1.0) / k * xk; xk *= x; }
        return s;
    }
    return log1p(x) - x / (1.0 + x);
}

/* 1 - ln(1+x)/x, regular at x -> 0 */
static double one_minus_log1p_over_x(double x)
{
    if (x < 1e-4) {   /* x/2 - x^2/3 + x^3/4 - ... */
        double s = 0.0, xk = x;
        for (int k = 2; k < 12; k++) { s += ((k & 1) ? -1.0 : 1.0) * xk / k; xk *= x; }
        return s;
    }
    return 1.0 - log1p(x) / x;
}

/* Velocity dispersion of the untruncated NFW halo with isotropic orbits
 * (reading: Lokas & Mamon's isotropic case, as the paper cites for sigma^2).
 * Isotropic Jeans equation: sigma^2(x) = 4 pi G rho_s r_s^2 x(1+x)^2 I(x),
 * I(x) = int_x^inf m(t) / (t^3 (1+t)^2) dt.  Computed by quadrature with the
 * substitution t = x/u, u in (0,1]. */
static double jeans_integrand(double u, void *vctx)
{
    double x = *(double *)vctx;
    double t = x / u;
    return orc_m(t) * u * u * u / (x * x * (u + x) * (u + x));
}

double orc_jeans_I_quad(double x)
{
    return quad(jeans_integrand, &x, 0.0, 1.0, 1e-14, 0.0);
}

/* Dilogarithm Li2(-x), x >= 0, for the closed-form cross-check only. */
static double li2_series(double w)  /* sum w^k/k^2, 0 <= w <= 1/2 */
{
    double s = 0.0, wk = w;
    for (int k = 1; k < 200; k++) { double t = wk / ((double)k * k); s += t; if (t < 1e-18 * s) break; wk *= w; }
    return s;
}
double orc_li2_neg(double x)
{
    if (x == 0.0) return 0.0;
    if (x > 1.0) {   /* inversion: Li2(-x) = -pi^2/6 - ln^2(x)/2 - Li2(-1/x) */
        double l = log(x);
        return -ORC_PI * ORC_PI / 6.0 - 0.5 * l * l - orc_li2_neg(1.0 / x);
    }
    /* Landen: Li2(z) = -Li2(z/(z-1)) - ln^2(1-z)/2 for z = -x <= 0 */
    double w = x / (1.0 + x), l = log1p(x);
    return -li2_series(w) - 0.5 * l * l;
}

/* Closed form of I(x) (Lokas & Mamon isotropic dispersion), used only as a
 * cross-check of the quadrature above. */
double orc_jeans_I_closed(double x)
{
    double l1 = log1p(x), ix = 1.0 / x, ip = 1.0 / (1.0 + x);
    return 0.5 * (ORC_PI * ORC_PI - log(x) - ix - ip * ip - 6.0 * ip
                  + (1.0 + ix * ix - 4.0 * ix - 2.0 * ip) * l1
                  + 3.0 * l1 * l1 + 6.0 * orc_li2_neg(x));
}

/* halo structural state shared by the energy integrands (CGS) */
struct halo_cgs {
    double c, rs, rho_s, M0, Mvir, rvir, V2, fb;
};

static double sigma2_cgs(const struct halo_cgs *h, double x)
{
    return 4.0 * ORC_PI * ORC_G * h->rho_s * h->rs * h->rs * x * (1.0 + x) * (1.0 + x) * orc_jeans_I_quad(x);
}

/* Potential of the NFW halo truncated at r_vir, zero at infinity (Sec. 2.1
 * footnote; reading: -G M_vir / r outside r_vir). */
static double phi_trunc(const struct halo_cgs *h, double r)
{
    if (r >= h->rvir) return -ORC_G * h->Mvir / r;
    double x = r / h->rs;
    double lx = (x < 1e-4) ? 1.0 - one_minus_log1p_over_x(x) : log1p(x) / x;
    return -ORC_G * h->M0 / h->rs * (lx - 1.0 / (1.0 + h->c));
}

/* kinetic part of Eq. initial_energy: 2 pi rho_tot 3 sigma^2 r^2, in x = r/r_s */
static double kin_integrand(double x, void *vctx)
{
    const struct halo_cgs *h = (const struct halo_cgs *)vctx;
    double rho = h->rho_s / (x * (1.0 + x) * (1.0 + x));
    double r = x * h->rs;
    return 2.0 * ORC_PI * rho * 3.0 * sigma2_cgs(h, x) * r * r * h->rs;
}
/* potential part of Eq. initial_energy: Phi dM/dr (no factor 1/2, as printed) */
static double pot_integrand(double x, void *vctx)
{
    const struct halo_cgs *h = (const struct halo_cgs *)vctx;
    double r = x * h->rs;
    double dMdx = h->M0 * x / ((1.0 + x) * (1.0 + x));
    return phi_trunc(h, r) * dMdx;
}

/* E over [x_lo, c] without the baryon-fraction factor */
static double energy_quad(const struct halo_cgs *h, double x_lo)
{
    double K = quad(kin_integrand, (void *)h, x_lo, h->c, 1e-12, 0.0);
    double W = quad(pot_integrand, (void *)h, x_lo, h->c, 1e-12, 0.0);
    return K + W;
}

/* Same energy by integration by parts with the Jeans equation (kinetic) and
 * elementary antiderivatives (potential) -- cross-check only. */
static double energy_closed(const struct halo_cgs *h, double x_lo)
{
    double c = h->c, G = ORC_G, M0 = h->M0, rs = h->rs;
    double A = G * M0 * M0 / rs;
    /* kinetic: (3/2)[4 pi r^3 rho sigma^2 / 3] + (1/2) G M0^2/r_s [-ln(1+x)/(1+x) - 1/(2(1+x)^2)] */
    double bnd_hi, bnd_lo;
    {
        double x = c, r = x * rs, rho = h->rho_s / (x * (1 + x) * (1 + x));
        bnd_hi = 4.0 * ORC_PI * r * r * r * rho * sigma2_cgs(h, x) / 3.0;
    }
    if (x_lo > 0) {
        double x = x_lo, r = x * rs, rho = h->rho_s / (x * (1 + x) * (1 + x));
        bnd_lo = 4.0 * ORC_PI * r * r * r * rho * sigma2_cgs(h, x) / 3.0;
    } else bnd_lo = 0.0;
#define KPRIM(x) (-log1p(x) / (1.0 + (x)) - 0.5 / ((1.0 + (x)) * (1.0 + (x))))
#define WPRIM(x) (-log1p(x) / (1.0 + (x)) - 1.0 / (1.0 + (x)) - orc_m(x) / (1.0 + c))
    double K = 1.5 * ((bnd_hi - bnd_lo) + A / 3.0 * (KPRIM(c) - KPRIM(x_lo)));
    double W = -A * (WPRIM(c) - WPRIM(x_lo));
#undef KPRIM
#undef WPRIM
    return K + W;
}

/* ======================================================================== */
/* Polytropic gas and boundary conditions (Sec. 2.1, 2.2).                   */
/* Reading: polytropic index n = 1/(Gamma-1) (the printed 1/Gamma - 1 is     */
/* inconsistent with P ~ rho^Gamma).  theta = 1 - a phi with                 */
/* a = ((Gamma-1)/Gamma)(rho0/P0) V^2 and phi = (Phi - Phi0)/V^2, V^2 = GM/r_vir. */
/* ======================================================================== */
struct gas_ctx {
    const orc_params *p;
    struct halo_cgs h;
    double npoly;          /* 1/(Gamma-1) */
    double phi0;           /* Phi0 [cgs] */
    double P_s, M_star_g, E_gi, E_DM;
    double a;              /* current trial slope */
    double x_f;            /* current trial r_f/r_vir */
    int kind;              /* integrand selector */
};

/* dimensionless potential above the centre, (Phi - Phi0)/V^2 */
static double phi_dimless(const struct gas_ctx *g, double r)
{
    const struct halo_cgs *h = &g->h;
    double c = h->c, mc = orc_m(c);
    if (r >= h->rvir) return c * c / ((1.0 + c) * mc) - h->rvir / r;
    return c / mc * one_minus_log1p_over_x(r / h->rs);
}

static double theta_of(const struct gas_ctx *g, double r)
{
    return 1.0 - g->a * phi_dimless(g, r);
}

/* integrands over r [cm] */
static double gas_integrand(double r, void *vctx)
{
    const struct gas_ctx *g = (const struct gas_ctx *)vctx;
    double th = theta_of(g, r);
    if (th <= 0.0) return 0.0;
    double w = 4.0 * ORC_PI * r * r;
    double thn = pow(th, g->npoly);
    if (g->kind == 0) return w * thn;                         /* gas-mass shape      */
    if (g->kind == 1) return w * thn * th;                    /* pressure shape      */
    /* kind 2: rho-shape times absolute potential */
    struct halo_cgs hh = g->h;
    return w * thn * phi_trunc(&hh, r);
}

static double gas_quad(struct gas_ctx *g, int kind, double r_f)
{
    g->kind = kind;
    double rv = g->h.rvir;
    if (r_f <= rv) return quad(gas_integrand, g, 0.0, r_f, 1e-13, 0.0);
    return quad(gas_integrand, g, 0.0, rv, 1e-13, 0.0) + quad(gas_integrand, g, rv, r_f, 1e-13, 0.0);
}

/* Gas-mass condition (Eq. gas_mass) fixes rho0, the definition of a fixes P0. */
static void rho0_P0(struct gas_ctx *g, double r_f, double *rho0, double *P0)
{
    double fbM = g->h.fb * g->h.Mvir;
    double I = gas_quad(g, 0, r_f);
    *rho0 = (fbM - g->M_star_g) / I;
    double Gm = g->p->Gamma;
    *P0 = (Gm - 1.0) / Gm * (*rho0) * g->h.V2 / g->a;
}

/* relative residual of the surface-pressure condition (Eq. surface_pressure) at trial a */
static double pressure_residual(double a, void *vctx)
{
    struct gas_ctx *g = (struct gas_ctx *)vctx;
    g->a = a;
    double r_f = g->x_f * g->h.rvir, rho0, P0;
    rho0_P0(g, r_f, &rho0, &P0);
    double th = theta_of(g, r_f);
    return P0 * pow(th, g->npoly + 1.0) / g->P_s - 1.0;
}

/* for a trial x_f: the slope a that satisfies the pressure condition */
static double solve_a(struct gas_ctx *g)
{
    double r_f = g->x_f * g->h.rvir;
    double a_max = 1.0 / phi_dimless(g, r_f);           /* theta(r_f) -> 0 */
    double lo = a_max * 1e-9, hi = a_max;
    double flo = pressure_residual(lo, g);
    double fhi = -1.0;                                  /* theta(r_f) = 0 exactly */
    if (!(flo > 0)) return NAN;
    return brent(pressure_residual, g, lo, hi, flo, fhi, 1e-16 * a_max, 300);
}

/* energy of the gas after rearrangement, E_gf = int 4 pi r^2 [3/2 P + rho Phi] dr */
static double gas_energy_final(struct gas_ctx *g, double r_f, double rho0, double P0)
{
    double Ip = gas_quad(g, 1, r_f);
    double Iphi = gas_quad(g, 2, r_f);
    return 1.5 * P0 * Ip + rho0 * Iphi;
}

/* relative residual of the energy condition (Eq. energy_conservation) at trial x_f.
 * Reading (energy_sign = 0): E_gf = E_gi + eps_DM|E_DM| + eps_* M_* c^2 + dE_p,
 * i.e. injected energy raises the gas energy.  energy_sign = 1 keeps the
 * printed arrangement E_gi = E_gf + eps_DM|E_DM| + eps_* M_* c^2 + dE_p. */
static double energy_residual(double x_f, void *vctx)
{
    struct gas_ctx *g = (struct gas_ctx *)vctx;
    g->x_f = x_f;
    double a = solve_a(g);
    if (!(a > 0)) return NAN;
    g->a = a;
    double r_f = x_f * g->h.rvir, rho0, P0;
    rho0_P0(g, r_f, &rho0, &P0);
    double Egf = gas_energy_final(g, r_f, rho0, P0);
    const orc_params *p = g->p;
    double rv = g->h.rvir;
    double dEp = 4.0 * ORC_PI / 3.0 * (rv * rv * rv - r_f * r_f * r_f) * g->P_s;
    double inj = p->eps_DM * fabs(g->E_DM) + p->eps_star * g->M_star_g * ORC_C * ORC_C;
    double res = (p->energy_sign == 0) ? Egf - (g->E_gi + inj + dEp) : g->E_gi - (Egf + inj + dEp);
    return res / fabs(g->E_gi);
}

/* ---- 1-D roots for r500 and r_* --------------------------------------- */
struct r500_ctx { double rho_s, target; };
static double r500_fn(double x, void *vctx)
{
    struct r500_ctx *cx = (struct r500_ctx *)vctx;
    return 3.0 * cx->rho_s * orc_m(x) / (x * x * x) - cx->target;
}
struct mstar_ctx { double target; };
static double mstar_fn(double x, void *vctx)
{
    return orc_m(x) - ((struct mstar_ctx *)vctx)->target;
}

/* Non-thermal pressure amplitude f(z) (Sec. 2.3) with f_max = 4^-n_nt / alpha_nt. */
double orc_f_nt(const orc_params *p, double z)
{
    double fmax = pow(4.0, -p->n_nt) / p->alpha_nt;
    double f1 = pow(1.0 + z, p->beta_nt);
    double f2 = (fmax - 1.0) * tanh(p->beta_nt * z) + 1.0;
    return fmin(f1, f2);
}

/* Number of x_f grid points scanned for a sign change of the energy residual. */
#define ORC_NSCAN 47
#define ORC_XF_LO 0.4
#define ORC_XF_HI 5.0

/* Solve the ICM model for one halo (M [Msun/h], c = r_vir/r_s, z). */
int orc_halo_solve(const orc_params *p, double M, double c, double z, orc_halo *o)
{
    memset(o, 0, sizeof(*o));
    o->M = M; o->c = c; o->z = z;
    if (!(M > 0) || !(c > 0) || !(z >= 0) || !isfinite(M) || !isfinite(c) || !isfinite(z)) {
        o->status = ORC_BAD_INPUT;
        return o->status;
    }
    const double h = p->h;
    /* --- halo structure (Sec. 2.1) --- */
    double E = hubble_E(p, z);
    double rho_crit = rho_crit0_hunits() * E * E;
    double Om_z = p->Omega_m * (1.0 + z) * (1.0 + z) * (1.0 + z) / (E * E);
    double xbn = Om_z - 1.0;
    /* reading: Bryan & Norman fit for flat universes, relative to rho_crit */
    double Dvir = 18.0 * ORC_PI * ORC_PI + 82.0 * xbn - 39.0 * xbn * xbn;
    double r_vir = cbrt(3.0 * M / (4.0 * ORC_PI * Dvir * rho_crit));
    double r_s = r_vir / c;
    double mc = orc_m(c);
    double rho_s = M / (4.0 * ORC_PI * r_s * r_s * r_s * mc);
    o->E = E; o->rho_crit = rho_crit; o->Delta_vir = Dvir;
    o->r_vir = r_vir; o->r_s = r_s; o->rho_s = rho_s;

    /* --- r500 (mean enclosed density 500 rho_crit) --- */
    struct r500_ctx rc = {rho_s, 500.0 * rho_crit};
    double xlo = c * 1e-8, xhi = c;
    double x500 = brent(r500_fn, &rc, xlo, xhi, r500_fn(xlo, &rc), r500_fn(xhi, &rc), 1e-15 * c, 300);
    o->x500 = x500; o->r500 = x500 * r_s;
    o->M500 = 4.0 * ORC_PI * rho_s * r_s * r_s * r_s * orc_m(x500);

    /* --- stars (Sec. 2.2); reading: the 3e14 Msun pivot has no h --- */
    double fb = p->Omega_b / p->Omega_m;
    o->F_star = p->f_star * pow(o->M500 / h / 3e14, -p->S_star);
    o->M_star = o->F_star * M;
    double ratio = o->M_star / (fb * M);
    if (!(ratio < 1.0)) { o->status = ORC_NO_STAR_ROOT; return o->status; }
    struct mstar_ctx mcx = {ratio * mc};
    o->x_star = brent(mstar_fn, &mcx, 0.0, c, -mcx.target, mc - mcx.target, 1e-15 * c, 300);

    /* --- CGS halo state --- */
    struct gas_ctx g;
    memset(&g, 0, sizeof(g));
    g.p = p;
    g.h.c = c;
    g.h.rs = r_s * ORC_MPC / h;
    g.h.rvir = r_vir * ORC_MPC / h;
    g.h.Mvir = M * ORC_MSUN / h;
    g.h.rho_s = rho_s * (ORC_MSUN / h) / pow(ORC_MPC / h, 3.0);
    g.h.M0 = 4.0 * ORC_PI * g.h.rho_s * g.h.rs * g.h.rs * g.h.rs;
    g.h.V2 = ORC_G * g.h.Mvir / g.h.rvir;
    g.h.fb = fb;
    g.npoly = 1.0 / (p->Gamma - 1.0);
    g.phi0 = -g.h.V2 * c * c / ((1.0 + c) * mc);
    g.M_star_g = o->M_star * ORC_MSUN / h;

    /* --- surface pressure (Eq. surface_pressure); reading: untruncated Jeans
     *     dispersion, NFW density just inside r_vir --- */
    o->sigma2_vir = sigma2_cgs(&g.h, c);
    double rho_vir = g.h.rho_s / (c * (1.0 + c) * (1.0 + c));
    g.P_s = fb * rho_vir * o->sigma2_vir;
    o->P_s = g.P_s;

    /* --- initial energies (Eq. initial_energy) --- */
    g.E_gi = fb * energy_quad(&g.h, o->x_star);
    g.E_DM = energy_quad(&g.h, 0.0);
    o->E_gi = g.E_gi; o->E_DM = g.E_DM;

    /* --- boundary-condition solve: scan x_f, Brent on the first sign change --- */
    double xs[ORC_NSCAN], rs_[ORC_NSCAN];
    int first = -1, nchg = 0;
    for (int i = 0; i < ORC_NSCAN; i++) {
        xs[i] = ORC_XF_LO + (ORC_XF_HI - ORC_XF_LO) * i / (ORC_NSCAN - 1);
        rs_[i] = energy_residual(xs[i], &g);
        if (!isfinite(rs_[i])) { o->status = ORC_NONFINITE; return o->status; }
        if (i > 0 && ((rs_[i - 1] < 0) != (rs_[i] < 0))) { nchg++; if (first < 0) first = i - 1; }
    }
    o->n_sign_changes = nchg;
    if (first < 0) { o->status = ORC_NO_BRACKET; return o->status; }
    if (nchg > 1) o->status |= ORC_MULTI_ROOT;
    double x_f = brent(energy_residual, &g, xs[first], xs[first + 1], rs_[first], rs_[first + 1],
                       1e-13 * xs[first], 200);
    o->res_E = energy_residual(x_f, &g);     /* also leaves g.a at the solution */
    double r_f = x_f * g.h.rvir, rho0, P0;
    rho0_P0(&g, r_f, &rho0, &P0);
    o->x_f = x_f; o->a = g.a; o->r_f = x_f * r_vir;
    o->rho0 = rho0; o->P0 = P0;
    o->res_P = P0 * pow(theta_of(&g, r_f), g.npoly + 1.0) / g.P_s - 1.0;
    o->res_M = (rho0 * gas_quad(&g, 0, r_f) + g.M_star_g) / (fb * g.h.Mvir) - 1.0;

    /* --- distances, optical depth, non-thermal pressure (Sec. 2.3, 3.2) --- */
    o->chi = orc_chi(p, z);
    o->D_A = o->chi / (1.0 + z);
    o->tau = orc_tau(p, z);
    o->f_nt = orc_f_nt(p, z);
    o->r_nt = o->r500 * pow(p->alpha_nt * o->f_nt, -1.0 / p->n_nt);
    o->R_t = fmin(o->r_f, p->trunc_r500 * o->r500);
    if (!isfinite(o->rho0) || !isfinite(o->P0) || !isfinite(o->x_f)) o->status |= ORC_NONFINITE;
    return o->status;
}

/* Cross-check entry points: energies by quadrature and in closed form for a
 * solved halo (lower limit x_lo in units of r_s; baryon fraction not applied). */
static void halo_cgs_of(const orc_params *p, const orc_halo *o, struct halo_cgs *hc)
{
    double h = p->h;
    hc->c = o->c;
    hc->rs = o->r_s * ORC_MPC / h;
    hc->rvir = o->r_vir * ORC_MPC / h;
    hc->Mvir = o->M * ORC_MSUN / h;
    hc->rho_s = o->rho_s * (ORC_MSUN / h) / pow(ORC_MPC / h, 3.0);
    hc->M0 = 4.0 * ORC_PI * hc->rho_s * hc->rs * hc->rs * hc->rs;
    hc->V2 = ORC_G * hc->Mvir / hc->rvir;
    hc->fb = p->Omega_b / p->Omega_m;
}
double orc_energy_quad(const orc_params *p, const orc_halo *o, double x_lo)
{
    struct halo_cgs hc; halo_cgs_of(p, o, &hc); return energy_quad(&hc, x_lo);
}
double orc_energy_closed(const orc_params *p, const orc_halo *o, double x_lo)
{
    struct halo_cgs hc; halo_cgs_of(p, o, &hc); return energy_closed(&hc, x_lo);
}
/* sigma^2 at x = r/r_s [cm^2/s^2] */
double orc_sigma2(const orc_params *p, const orc_halo *o, double x)
{
    struct halo_cgs hc; halo_cgs_of(p, o, &hc); return sigma2_cgs(&hc, x);
}
/* residual functions exposed for tests: relative residual of the energy and
 * pressure conditions at an arbitrary trial (x_f, a) */
double orc_energy_residual_at(const orc_params *p, const orc_halo *o, double x_f)
{
    struct gas_ctx g; memset(&g, 0, sizeof(g));
    g.p = p; halo_cgs_of(p, o, &g.h);
    g.npoly = 1.0 / (p->Gamma - 1.0);
    g.phi0 = -g.h.V2 * o->c * o->c / ((1.0 + o->c) * orc_m(o->c));
    g.P_s = o->P_s; g.M_star_g = o->M_star * ORC_MSUN / p->h;
    g.E_gi = o->E_gi; g.E_DM = o->E_DM;
    return energy_residual(x_f, &g);
}

/* ======================================================================== */
/* Gas profiles of a solved halo (Sec. 2.1, 2.3, 3.2).  r in physical Mpc/h. */
/* ======================================================================== */
struct prof_ctx {
    const orc_params *p;
    const orc_halo *o;
    struct gas_ctx g;
    double rperp2_cm;     /* impact parameter squared [cm^2] */
    int which;            /* 0: electron pressure, 1: electron density */
};

static void prof_init(struct prof_ctx *pc, const orc_params *p, const orc_halo *o)
{
    memset(pc, 0, sizeof(*pc));
    pc->p = p; pc->o = o;
    pc->g.p = p;
    halo_cgs_of(p, o, &pc->g.h);
    pc->g.npoly = 1.0 / (p->Gamma - 1.0);
    pc->g.a = o->a;
}

/* total gas pressure, gas density at r [cm]; zero outside r_f */
static void gas_at(const struct prof_ctx *pc, double r_cm, double *Ptot, double *rho_g)
{
    double rf = pc->o->r_f * ORC_MPC / pc->p->h;
    if (r_cm >= rf) { *Ptot = 0; *rho_g = 0; return; }
    double th = theta_of(&pc->g, r_cm);
    if (th <= 0) { *Ptot = 0; *rho_g = 0; return; }
    double thn = pow(th, pc->g.npoly);
    *Ptot = pc->o->P0 * thn * th;
    *rho_g = pc->o->rho0 * thn;
}

/* electron pressure [erg/cm^3] and electron number density [1/cm^3] at r.
 * P_th = P_tot max(0, 1 - R_nt), R_nt = alpha f(z) (r/r500)^n_nt;
 * P_e = (2X+2)/(5X+3) P_th; n_e = rho_g/(mu_e m_p), mu_e = 2/(1+X) (reading:
 * n_e of the halo gas is its fully ionised electron density). */
static void electrons_at(const struct prof_ctx *pc, double r_cm, double *Pe, double *ne)
{
    const orc_params *p = pc->p;
    double Ptot, rho;
    gas_at(pc, r_cm, &Ptot, &rho);
    double r500 = pc->o->r500 * ORC_MPC / p->h;
    double Rnt = p->alpha_nt * pc->o->f_nt * pow(r_cm / r500, p->n_nt);
    double Pth = Ptot * fmax(0.0, 1.0 - Rnt);
    double X = p->X_H;
    *Pe = (2.0 * X + 2.0) / (5.0 * X + 3.0) * Pth;
    *ne = rho / (2.0 / (1.0 + X) * ORC_MP);
}

void orc_profile(const orc_params *p, const orc_halo *o, double r_mpch, double *Pe, double *ne)
{
    struct prof_ctx pc; prof_init(&pc, p, o);
    electrons_at(&pc, r_mpch * ORC_MPC / p->h, Pe, ne);
}

static double los_integrand(double r, void *vctx)
{
    const struct prof_ctx *pc = (const struct prof_ctx *)vctx;
    double Pe, ne;
    electrons_at(pc, r, &Pe, &ne);
    return pc->which == 0 ? Pe : ne;
}

/* Sight line through a spherical profile f(r) at impact parameter rp, out to
 * the radius rmax where the profile ends (Sec. 3.3: each map value is the
 * integral of the gas quantity along the line of sight):
 *     2 int_0^sqrt(rmax^2 - rp^2) f(sqrt(rp^2 + l^2)) dl.
 * The line is split where it crosses any of the nr radii in (rp, rmax), so
 * that each piece has a smooth integrand (kinks of the profile). */
struct los_ctx { orc_fn f; void *ctx; double rp2; };
static double los_line(double l, void *vctx)
{
    const struct los_ctx *lc = (const struct los_ctx *)vctx;
    return lc->f(sqrt(lc->rp2 + l * l), lc->ctx);
}
static double los_integral(orc_fn f, void *ctx, double rp, double rmax, const double *radii, int nr)
{
    if (!(rp < rmax)) return 0.0;
    struct los_ctx lc = {f, ctx, rp * rp};
    double L = sqrt(rmax * rmax - rp * rp);
    double brk[10]; int nb = 0;
    brk[nb++] = 0.0;
    for (int k = 0; k < nr && k < 8; k++) {
        if (!(radii[k] > rp && radii[k] < rmax)) continue;
        double cut = sqrt(radii[k] * radii[k] - rp * rp);
        int j = nb;                               /* insertion keeps the cuts increasing */
        while (j > 1 && brk[j - 1] > cut) { brk[j] = brk[j - 1]; j--; }
        brk[j] = cut; nb++;
    }
    brk[nb++] = L;
    double s = 0.0;
    for (int k = 0; k + 1 < nb; k++) s += quad(los_line, &lc, brk[k], brk[k + 1], 1e-12, 0.0);
    return 2.0 * s;
}

/* Line-of-sight integrals through one halo at impact parameter r_perp (HP,
 * Sec. 3.3):  Y_P = 2 int_0^sqrt(r_f^2 - r_perp^2) P_e dl  and Y_n the same
 * with n_e.  Returned already multiplied by the observable prefactors:
 *   ty = sigma_T/(m_e c^2) Y_P        (the Compton-y contribution)
 *   tb = sigma_T Y_n                  (b contribution per unit v/c e^-tau)
 * The integral is split where the sight line crosses r_vir (kink of the
 * potential) and where R_nt reaches 1. */
void orc_los(const orc_params *p, const orc_halo *o, double rperp_mpch, double *ty, double *tb)
{
    struct prof_ctx pc; prof_init(&pc, p, o);
    double u = ORC_MPC / p->h;
    double rp = rperp_mpch * u, rf = o->r_f * u;
    double radii[2] = {o->r_vir * u, o->r_nt * u};
    pc.which = 0; double sy = los_integral(los_integrand, &pc, rp, rf, radii, 2);
    pc.which = 1; double sb = los_integral(los_integrand, &pc, rp, rf, radii, 2);
    *ty = ORC_SIGMA_T / ORC_ME_C2 * sy;
    *tb = ORC_SIGMA_T * sb;
}

/* Test entry point: the same sight-line integral through a model profile with
 * a known projection, so the integration itself is pinned by closed forms.
 *   kind 0: uniform sphere, f = 1 for r < rmax;
 *   kind 1: beta model, f = (1 + (r/rc)^2)^(-3 beta / 2), beta = par1, rc = par2;
 *   kind 2: two shells, f = 1 for r < par1, f = par2 for par1 <= r < rmax
 *           (a jump at par1, given to the integral as a split radius).
 * Lengths in any unit; returns 2 int f dl in that unit. */
static double model_profile(double r, void *vctx)
{
    const double *m = (const double *)vctx;   /* kind, par1, par2 */
    int kind = (int)m[0];
    if (kind == 0) return 1.0;
    if (kind == 1) return pow(1.0 + (r / m[2]) * (r / m[2]), -1.5 * m[1]);
    return r < m[1] ? 1.0 : m[2];
}
double orc_los_model(int kind, double par1, double par2, double rmax, double rp)
{
    double m[3] = {(double)kind, par1, par2};
    double radii[1] = {par1};
    return los_integral(model_profile, m, rp, rmax, radii, kind == 2 ? 1 : 0);
}

/* ======================================================================== */
/* HP flat-sky map (Sec. 3.3).  Pixel (i,j) of an npix x npix map of pixel   */
/* size pix_rad has centre ((i+1/2) pix, (j+1/2) pix); maps are row-major    */
/* [j][i].  Reading: the value of a pixel is the sight line through its      */
/* centre; the impact parameter is D_A |dtheta| on the tangent plane; a halo */
/* contributes where r_perp < R_t = min(r_f, trunc_r500 r500) (the cut acts  */
/* on the projected radius only).  Maps ACCUMULATE.                          */
/* ======================================================================== */
static void hp_flat_one(const orc_params *p, const orc_halo *o, double thx, double thy, double v_kms,
                        int npix, double pix, double *ymap, double *bmap)
{
    if (o->status & ~ORC_MULTI_ROOT) return;
    double ang_R = o->R_t / o->D_A;             /* footprint radius [rad] */
    int i0 = (int)floor((thx - ang_R) / pix) - 1, i1 = (int)floor((thx + ang_R) / pix) + 1;
    int j0 = (int)floor((thy - ang_R) / pix) - 1, j1 = (int)floor((thy + ang_R) / pix) + 1;
    if (i0 < 0) i0 = 0;
    if (j0 < 0) j0 = 0;
    if (i1 > npix - 1) i1 = npix - 1;
    if (j1 > npix - 1) j1 = npix - 1;
    double kb = v_kms * 1e5 / ORC_C * exp(-o->tau);
    for (int j = j0; j <= j1; j++)
        for (int i = i0; i <= i1; i++) {
            double dx = (i + 0.5) * pix - thx, dy = (j + 0.5) * pix - thy;
            double rp = o->D_A * sqrt(dx * dx + dy * dy);
            if (!(rp < o->R_t)) continue;
            double ty, tb;
            orc_los(p, o, rp, &ty, &tb);
            ymap[(int64_t)j * npix + i] += ty;
            bmap[(int64_t)j * npix + i] += kb * tb;
        }
}

/* Full HP flat map from a catalogue; halos[] (may be NULL) receives the solutions. */
int orc_hp_flat(const orc_params *p, int64_t n, const double *M, const double *c, const double *z,
                const double *thx, const double *thy, const double *v, int npix, double pix,
                double *ymap, double *bmap, orc_halo *halos)
{
    int nbad = 0;
    for (int64_t k = 0; k < n; k++) {
        orc_halo o;
        orc_halo_solve(p, M[k], c[k], z[k], &o);
        if (o.status & ~ORC_MULTI_ROOT) nbad++;
        hp_flat_one(p, &o, thx[k], thy[k], v[k], npix, pix, ymap, bmap);
        if (halos) halos[k] = o;
    }
    return nbad;
}

/* Same map but from halos already solved (halos[k] must correspond to thx[k]...). */
void orc_hp_flat_solved(const orc_params *p, int64_t n, const orc_halo *halos, const double *thx,
                        const double *thy, const double *v, int npix, double pix,
                        double *ymap, double *bmap)
{
    for (int64_t k = 0; k < n; k++) hp_flat_one(p, &halos[k], thx[k], thy[k], v[k], npix, pix, ymap, bmap);
}

/* Selected pixels only (for sampled parity on large maps): out_y[q], out_b[q]
 * receive the sum over all given halos at pixel (pi[q], pj[q]). */
void orc_hp_flat_pixels(const orc_params *p, int64_t n, const orc_halo *halos, const double *thx,
                        const double *thy, const double *v, double pix, int64_t nq,
                        const int32_t *pi, const int32_t *pj, double *out_y, double *out_b)
{
    for (int64_t q = 0; q < nq; q++) { out_y[q] = 0; out_b[q] = 0; }
    for (int64_t k = 0; k < n; k++) {
        const orc_halo *o = &halos[k];
        if (o->status & ~ORC_MULTI_ROOT) continue;
        double kb = v[k] * 1e5 / ORC_C * exp(-o->tau);
        for (int64_t q = 0; q < nq; q++) {
            double dx = (pi[q] + 0.5) * pix - thx[k], dy = (pj[q] + 0.5) * pix - thy[k];
            double rp = o->D_A * sqrt(dx * dx + dy * dy);
            if (!(rp < o->R_t)) continue;
            double ty, tb;
            orc_los(p, o, rp, &ty, &tb);
            out_y[q] += ty;
            out_b[q] += kb * tb;
        }
    }
}

/* ======================================================================== */
/* HEALPix RING pixelisation (Gorski et al. 2005, the scheme the paper's     */
/* all-sky maps use).  Rings i = 1..4N-1 from the north pole; the polar caps */
/* have 4i pixels per ring, the equatorial belt 4N.  Written from the        */
/* geometry: in the belt pixel edges are the lines t -+ (3/4) z = const with */
/* t = 2 phi / pi; in the caps they are t_frac * N sqrt(3(1-|z|)) = const.   */
/* Floating-point steps are kept in a fixed order (no contraction) so that   */
/* the integer result is reproducible bit for bit.                           */
/* ======================================================================== */
/* Reading: the pixel of a direction is the one its cos(theta) and sin(theta), rounded correctly to
 * FP64, select.  Next to a pixel edge the last bit of either decides the index, and libm's cos and sin
 * are not always correctly rounded; here both are evaluated in quad precision and rounded once. */
static double cos_cr(double t) { return (double)cosq((__float128)t); }
static double sin_cr(double t) { return (double)sinq((__float128)t); }

int64_t orc_ang2pix_ring(int64_t nside, double theta, double phi)
{
    const double halfpi = 1.5707963267948966;
    double z = cos_cr(theta), za = fabs(z);
    double tt = phi / halfpi;                     /* in [0,4) for phi in [0,2pi) */
    tt = tt - 4.0 * floor(tt / 4.0);
    if (tt >= 4.0) tt = 0.0;
    int64_t N = nside;
    if (za <= 2.0 / 3.0) {
        double a = (double)N * (0.5 + tt);
        double b = (double)N * (z * 0.75);
        int64_t asc = (int64_t)floor(a - b);      /* ascending edge-line index  */
        int64_t dsc = (int64_t)floor(a + b);      /* descending edge-line index */
        int64_t ir = N + 1 + asc - dsc;           /* 1..2N+1, counted from z = 2/3 */
        int64_t odd = 1 - (ir & 1);
        int64_t ip = (asc + dsc - N + odd + 1) / 2;
        ip = ((ip % (4 * N)) + 4 * N) % (4 * N);
        return 2 * N * (N - 1) + (ir - 1) * 4 * N + ip;
    }
    double tf = tt - floor(tt);
    double s = sin_cr(theta);
    double tmp = (double)N * (s * sqrt(3.0 / (1.0 + za)));   /* = N sqrt(3(1-|z|)) */
    int64_t jp = (int64_t)floor(tf * tmp);
    int64_t jm = (int64_t)floor((1.0 - tf) * tmp);
    int64_t ir = jp + jm + 1;                                 /* ring from the pole */
    int64_t ip = (int64_t)floor(tt * (double)ir);
    ip = ((ip % (4 * ir)) + 4 * ir) % (4 * ir);
    if (z > 0) return 2 * ir * (ir - 1) + ip;
    return 12 * N * N - 2 * ir * (ir + 1) + ip;
}

static int64_t isqrt64(int64_t v)
{
    int64_t r = (int64_t)sqrt((double)v);
    while (r * r > v) r--;
    while ((r + 1) * (r + 1) <= v) r++;
    return r;
}

/* Ring index (1..4N-1) and position j (1..npix in ring) of a RING pixel. */
static void ring_of(int64_t N, int64_t p, int64_t *ring, int64_t *j)
{
    int64_t ncap = 2 * N * (N - 1), npix = 12 * N * N;
    if (p < ncap) {
        int64_t i = (1 + isqrt64(1 + 2 * p)) / 2;
        while (2 * i * (i - 1) > p) i--;
        while (2 * (i + 1) * i <= p) i++;
        *ring = i; *j = p - 2 * i * (i - 1) + 1;
    } else if (p < npix - ncap) {
        int64_t q = p - ncap;
        *ring = q / (4 * N) + N; *j = q % (4 * N) + 1;
    } else {
        int64_t q = npix - 1 - p;           /* mirror of the north cap */
        int64_t i = (1 + isqrt64(1 + 2 * q)) / 2;
        while (2 * i * (i - 1) > q) i--;
        while (2 * (i + 1) * i <= q) i++;
        int64_t jj = q - 2 * i * (i - 1) + 1;  /* counted backwards */
        *ring = 4 * N - i; *j = 4 * i - jj + 1;
    }
}

/* Centre of a RING pixel: colatitude theta, longitude phi. */
void orc_pix2ang_ring(int64_t nside, int64_t p, double *theta, double *phi)
{
    int64_t N = nside, ring, j;
    ring_of(N, p, &ring, &j);
    const double halfpi = 1.5707963267948966;
    if (ring < N) {                                   /* north cap */
        double i = (double)ring;
        *theta = 2.0 * asin(i / (sqrt(6.0) * (double)N));
        *phi = halfpi / i * ((double)j - 0.5);
    } else if (ring <= 3 * N) {                       /* belt */
        double z = (double)(2 * N - ring) * 2.0 / (3.0 * (double)N);
        *theta = acos(z);
        double shift = ((ring + N) & 1) ? 1.0 : 0.5;
        *phi = halfpi / (double)N * ((double)j - shift);
    } else {                                          /* south cap */
        double i = (double)(4 * N - ring);
        *theta = ORC_PI - 2.0 * asin(i / (sqrt(6.0) * (double)N));
        *phi = halfpi / i * ((double)j - 0.5);
    }
}

/* HP all-sky map on HEALPix RING pixels.  Reading: the impact parameter is
 * D_A sin(psi) with psi the angle between the pixel centre and the halo
 * centre (psi < pi/2); a halo contributes where r_perp < R_t.  Brute force
 * over all pixels: small nside only.  Maps ACCUMULATE. */
int orc_hp_healpix(const orc_params *p, int64_t n, const double *M, const double *c, const double *z,
                   const double *th, const double *ph, const double *v, int64_t nside,
                   double *ymap, double *bmap, orc_halo *halos)
{
    int64_t npix = 12 * nside * nside;
    double *px = malloc(sizeof(double) * npix), *py = malloc(sizeof(double) * npix),
           *pz = malloc(sizeof(double) * npix);
    for (int64_t q = 0; q < npix; q++) {
        double t, f;
        orc_pix2ang_ring(nside, q, &t, &f);
        px[q] = sin(t) * cos(f); py[q] = sin(t) * sin(f); pz[q] = cos(t);
    }
    int nbad = 0;
    for (int64_t k = 0; k < n; k++) {
        orc_halo o;
        orc_halo_solve(p, M[k], c[k], z[k], &o);
        if (halos) halos[k] = o;
        if (o.status & ~ORC_MULTI_ROOT) { nbad++; continue; }
        double hx = sin(th[k]) * cos(ph[k]), hy = sin(th[k]) * sin(ph[k]), hz = cos(th[k]);
        double kb = v[k] * 1e5 / ORC_C * exp(-o.tau);
        for (int64_t q = 0; q < npix; q++) {
            double dot = px[q] * hx + py[q] * hy + pz[q] * hz;
            if (!(dot > 0)) continue;
            double cx = py[q] * hz - pz[q] * hy, cy = pz[q] * hx - px[q] * hz, cz = px[q] * hy - py[q] * hx;
            double sinpsi = sqrt(cx * cx + cy * cy + cz * cz);
            double rp = o.D_A * sinpsi;
            if (!(rp < o.R_t)) continue;
            double ty, tb;
            orc_los(p, &o, rp, &ty, &tb);
            ymap[q] += ty;
            bmap[q] += kb * tb;
        }
    }
    free(px); free(py); free(pz);
    return nbad;
}

/* Selected HEALPix pixels only, from solved halos. */
void orc_hp_healpix_pixels(const orc_params *p, int64_t n, const orc_halo *halos, const double *th,
                           const double *ph, const double *v, int64_t nside, int64_t nq,
                           const int64_t *pix, double *out_y, double *out_b)
{
    for (int64_t q = 0; q < nq; q++) {
        out_y[q] = 0; out_b[q] = 0;
        double t, f;
        orc_pix2ang_ring(nside, pix[q], &t, &f);
        double px = sin(t) * cos(f), py = sin(t) * sin(f), pz = cos(t);
        for (int64_t k = 0; k < n; k++) {
            const orc_halo *o = &halos[k];
            if (o->status & ~ORC_MULTI_ROOT) continue;
            double hx = sin(th[k]) * cos(ph[k]), hy = sin(th[k]) * sin(ph[k]), hz = cos(th[k]);
            double dot = px * hx + py * hy + pz * hz;
            if (!(dot > 0)) continue;
            double cx = py * hz - pz * hy, cy = pz * hx - px * hz, cz = px * hy - py * hx;
            double rp = o->D_A * sqrt(cx * cx + cy * cy + cz * cz);
            if (!(rp < o->R_t)) continue;
            double ty, tb;
            orc_los(p, o, rp, &ty, &tb);
            out_y[q] += ty;
            out_b[q] += v[k] * 1e5 / ORC_C * exp(-o->tau) * tb;
        }
    }
}

/* ======================================================================== */
/* PP: particle-based pasting (Sec. 3.4).                                    */
/* ======================================================================== */
/* Cubic-spline kernel shape of Eq. SPH_kernel without the 8/(pi h^3) factor */
double orc_W_sph(double x)
{
    x = fabs(x);
    if (x < 0.5) return 1.0 - 6.0 * x * x + 6.0 * x * x * x;
    if (x < 1.0) return 2.0 * (1.0 - x) * (1.0 - x) * (1.0 - x);
    return 0.0;
}

/* Normalised integral of the kernel along one axis, Eq. integrated_kernel */
double orc_w_sph(double x)
{
    if (x < -1.0) return 0.0;
    if (x <= -0.5) return 2.0 / 3.0 * pow(1.0 + x, 4);
    if (x <= 0.0) return 4.0 / 3.0 * (0.375 + x - 2.0 * x * x * x - 1.5 * x * x * x * x);
    if (x <= 0.5) return 4.0 / 3.0 * (0.375 + x - 2.0 * x * x * x + 1.5 * x * x * x * x);
    if (x <= 1.0) return -2.0 / 3.0 * pow(1.0 - x, 4) + 1.0;
    return 1.0;
}

/* Smoothing length: distance to the k-th nearest OTHER particle in 3-D
 * comoving Cartesian coordinates (reading of the paper's neighbour-number
 * criterion for a fixed neighbour count).  Brute force, O(n^2): small n. */
static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}
void orc_knn_h(int64_t n, const double *X, const double *Y, const double *Z, int k, double *h)
{
    double *d = malloc(sizeof(double) * (n > 1 ? n - 1 : 1));
    for (int64_t i = 0; i < n; i++) {
        int64_t m = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
            d[m++] = dx * dx + dy * dy + dz * dz;
        }
        if (m < k) { h[i] = NAN; continue; }
        qsort(d, m, sizeof(double), cmp_double);
        h[i] = sqrt(d[k - 1]);
    }
    free(d);
}

/* The same smoothing length for a subset of the points only (qidx[a] indexes
 * X, Y, Z): brute force over all n points for each query.  For checks on
 * samples of large particle sets, given every point that can be a neighbour. */
void orc_knn_h_query(int64_t nq, const int64_t *qidx, int64_t n, const double *X, const double *Y,
                     const double *Z, int k, double *h)
{
    double *d = malloc(sizeof(double) * (n > 1 ? n - 1 : 1));
    for (int64_t a = 0; a < nq; a++) {
        int64_t i = qidx[a], m = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
            d[m++] = dx * dx + dy * dy + dz * dz;
        }
        if (m < k) { h[a] = NAN; continue; }
        qsort(d, m, sizeof(double), cmp_double);
        h[a] = sqrt(d[k - 1]);
    }
    free(d);
}

/* Smoothing length from the effective neighbour number (Sec. 3.4, with the
 * cubic-spline kernel of Eq. SPH_kernel): h solves
 *     N_eff(h) = (4 pi / 3) h^3 sum_j W(r_ij, h) = n_ngb,
 * W = 8/(pi h^3) orc_W_sph(r/h).  reading: the sum runs over every particle,
 * the particle itself included (the standard SPH density estimate), so that
 * N_eff(h) = (32/3) sum_j orc_W_sph(r_ij / h).  N_eff is continuous and
 * non-decreasing in h; the root is found by bisection on the sorted distances
 * of every point to the query (brute force, O(n log n) per query).  NaN when
 * even all n points cannot reach n_ngb ((32/3) n <= n_ngb). */
static double neff_sum(const double *d, int64_t m, double h)
{
    double s = 0.0;
    for (int64_t j = 0; j < m && d[j] < h; j++) s += orc_W_sph(d[j] / h);
    return 32.0 / 3.0 * s;
}
void orc_neff_h_query(int64_t nq, const int64_t *qidx, int64_t n, const double *X, const double *Y,
                      const double *Z, double n_ngb, double *h)
{
    double *d = malloc(sizeof(double) * (n > 0 ? n : 1));
    for (int64_t a = 0; a < nq; a++) {
        int64_t i = qidx[a];
        for (int64_t j = 0; j < n; j++) {
            double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
            d[j] = sqrt(dx * dx + dy * dy + dz * dz);
        }
        qsort(d, n, sizeof(double), cmp_double);
        /* N_eff rises to (32/3) n as h grows: no root unless that exceeds n_ngb; otherwise
         * double the upper end from twice the largest distance until it brackets the root */
        if (32.0 / 3.0 * (double)n <= n_ngb) { h[a] = NAN; continue; }
        double lo = 0.0, hi = 2.0 * d[n - 1] + 1e-300;
        while (neff_sum(d, n, hi) < n_ngb) hi *= 2.0;
        for (int it = 0; it < 400 && hi - lo > 1e-15 * hi; it++) {
            double mid = 0.5 * (lo + hi);
            if (neff_sum(d, n, mid) < n_ngb) lo = mid; else hi = mid;
        }
        h[a] = 0.5 * (lo + hi);
    }
    free(d);
}

/* N_eff(h) of one point: the quantity the smoothing length sets to n_ngb. */
double orc_neff_at(int64_t n, const double *X, const double *Y, const double *Z, int64_t i, double h)
{
    double s = 0.0;
    for (int64_t j = 0; j < n; j++) {
        double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
        s += orc_W_sph(sqrt(dx * dx + dy * dy + dz * dz) / h);
    }
    return 32.0 / 3.0 * s;
}

/* Per-particle signal amplitudes (Sec. 3.4).
 * Halo particle (halo_id >= 0):
 *   y_i = sigma_T/(m_e c^2) P_e(r_i) V_i / L_pix^2,
 *   b_i = sigma_T (v_i/c) e^-tau_i n_e(r_i) V_i / L_pix^2,
 *   V_i = M_p / rho_tot(r_i) with the untruncated NFW density (reading),
 *   P_e = n_e = 0 for r_i >= r_f.
 * Field particle (halo_id < 0):
 *   y_i = 0,  b_i = sigma_T (v_i/c) (f_gas M_p / (mu_e m_p)) e^-tau_i / L_pix^2
 *   (reading: f_gas = field_gas_frac, default the cosmic baryon fraction).
 *   With field_T > 0 the field gas carries the pressure P_e = n_e k_B T (the filament extension
 *   that Sec. 3.4 leaves open; reading: electrons at the gas temperature, and, like the halo tSZ
 *   term, no e^-tau):  y_i = sigma_T/(m_e c^2) k_B T (f_gas M_p / (mu_e m_p)) / L_pix^2.
 * L_pix = D_A(z_i) pix is the physical pixel size at the particle.
 * Inputs: z_i, v_i [km/s], r_i [physical Mpc/h], M_p [Msun/h]. */
void orc_pp_amplitudes(const orc_params *p, int64_t n, const double *zp, const double *v,
                       const int32_t *halo_id, const double *r_i, double M_p, double pix,
                       const orc_halo *halos, double *amp_y, double *amp_b)
{
    double u = ORC_MPC / p->h, Mp_g = M_p * ORC_MSUN / p->h;
    double mu_e = 2.0 / (1.0 + p->X_H);
    for (int64_t i = 0; i < n; i++) {
        double DA = orc_DA(p, zp[i]) * u;
        double Lpix = DA * pix;
        double ek = exp(-orc_tau(p, zp[i]));
        double vc = v[i] * 1e5 / ORC_C;
        if (halo_id[i] < 0) {
            double Ne = p->field_gas_frac * Mp_g / (mu_e * ORC_MP);
            amp_y[i] = ORC_SIGMA_T / ORC_ME_C2 * (ORC_KB * p->field_T) * Ne / (Lpix * Lpix);
            amp_b[i] = ORC_SIGMA_T * vc * Ne * ek / (Lpix * Lpix);
            continue;
        }
        const orc_halo *o = &halos[halo_id[i]];
        if (o->status & ~ORC_MULTI_ROOT) { amp_y[i] = 0; amp_b[i] = 0; continue; }
        double x = r_i[i] / o->r_s;
        double rho_s_cgs = o->rho_s * (ORC_MSUN / p->h) / (u * u * u);
        double rho_tot = rho_s_cgs / (x * (1.0 + x) * (1.0 + x));
        double V = Mp_g / rho_tot;
        double Pe, ne;
        orc_profile(p, o, r_i[i], &Pe, &ne);
        amp_y[i] = ORC_SIGMA_T / ORC_ME_C2 * Pe * V / (Lpix * Lpix);
        amp_b[i] = ORC_SIGMA_T * vc * ek * ne * V / (Lpix * Lpix);
    }
}

/* SPH deposit on the flat map (Sec. 3.4): every pixel (i,j) overlapping the
 * particle's 2H square receives amp * f_ij with
 *   f_ij = [w((x_i^+ - x_p)/H) - w((x_i^- - x_p)/H)] [same in y],
 * pixel edges x_i^- = i pix, x_i^+ = (i+1) pix.  H = h_comoving / chi is the
 * angular smoothing length.  Reading: pixels outside the map are dropped,
 * with no renormalisation.  Maps ACCUMULATE. */
void orc_pp_deposit(int64_t n, const double *thx, const double *thy, const double *H,
                    const double *amp_y, const double *amp_b, int npix, double pix,
                    double *ymap, double *bmap)
{
    for (int64_t k = 0; k < n; k++) {
        double Hk = H[k];
        int i0 = (int)floor((thx[k] - Hk) / pix), i1 = (int)floor((thx[k] + Hk) / pix);
        int j0 = (int)floor((thy[k] - Hk) / pix), j1 = (int)floor((thy[k] + Hk) / pix);
        if (i0 < 0) i0 = 0;
        if (j0 < 0) j0 = 0;
        if (i1 > npix - 1) i1 = npix - 1;
        if (j1 > npix - 1) j1 = npix - 1;
        for (int j = j0; j <= j1; j++) {
            double fy = orc_w_sph(((j + 1) * pix - thy[k]) / Hk) - orc_w_sph((j * pix - thy[k]) / Hk);
            for (int i = i0; i <= i1; i++) {
                double fx = orc_w_sph(((i + 1) * pix - thx[k]) / Hk) - orc_w_sph((i * pix - thx[k]) / Hk);
                double f = fx * fy;
                ymap[(int64_t)j * npix + i] += amp_y[k] * f;
                bmap[(int64_t)j * npix + i] += amp_b[k] * f;
            }
        }
    }
}

/* All-sky particle kSZ by nearest-pixel assignment (App. A, continuous light cone):
 * every particle is a field particle (Eq. field_b, field_y) and its whole amplitude goes to
 * one HEALPix RING pixel.
 * Reading: the nearest pixel is the pixel that contains the particle's direction (the
 * HEALPix ang2pix assignment), and the pixel area at the particle is L_pix^2 = D_A^2 Omega_pix
 * with the equal pixel solid angle Omega_pix = 4 pi / (12 N_side^2).
 * Outputs per particle: pix[i] (RING index, -1 for a colatitude outside [0, pi] or a
 * non-finite angle, which then deposits nothing) and amp[i] = b_i. */
void orc_pp_healpix_ngp(const orc_params *p, int64_t n, const double *theta, const double *phi,
                        const double *zp, const double *v, double M_p, int64_t nside,
                        int64_t *pix, double *amp)
{
    double omega_pix = 4.0 * ORC_PI / (12.0 * (double)nside * (double)nside);
    int32_t field = -1;
    double zero = 0.0, ay;
    for (int64_t i = 0; i < n; i++) {
        int ok = theta[i] >= 0.0 && theta[i] <= ORC_PI && isfinite(phi[i]);
        pix[i] = ok ? orc_ang2pix_ring(nside, theta[i], phi[i]) : -1;
        orc_pp_amplitudes(p, 1, &zp[i], &v[i], &field, &zero, M_p, sqrt(omega_pix), NULL, &ay, &amp[i]);
        if (!ok) amp[i] = 0.0;
    }
}

/* The map itself: b_map[pix] += b_i in particle order (b_map has 12 N_side^2 entries and
 * ACCUMULATES); babs_map (may be NULL) receives sum |b_i| per pixel, the scale of the
 * rounding error of any summation order. */
void orc_pp_healpix_ngp_map(const orc_params *p, int64_t n, const double *theta, const double *phi,
                            const double *zp, const double *v, double M_p, int64_t nside,
                            double *b_map, double *babs_map)
{
    int64_t *pix = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    double *amp = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    orc_pp_healpix_ngp(p, n, theta, phi, zp, v, M_p, nside, pix, amp);
    for (int64_t i = 0; i < n; i++) {
        if (pix[i] < 0) continue;
        b_map[pix[i]] += amp[i];
        if (babs_map) babs_map[pix[i]] += fabs(amp[i]);
    }
    free(pix);
    free(amp);
}

/* size of orc_halo for the binding to check its mirror */
int orc_sizeof_halo(void) { return (int)sizeof(orc_halo); }
int orc_sizeof_params(void) { return (int)sizeof(orc_params); }
