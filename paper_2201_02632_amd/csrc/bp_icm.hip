// K1 (ICM boundary-condition solve) and K2 (projected profile tables).
//
// K1: one lane per halo, FP64 (Sec. 2 of Osato & Nagai 2022).  For a trial
// gas boundary x_f = r_f/r_vir the polytrope integrals are polynomials in the
// slope a, since theta = 1 - a phi(r):
//     int 4 pi r^2 theta^n dr = sum_k C(n,k) (-a)^k mu_k,   mu_k = int 4 pi r^2 phi^k dr
// so each x_f costs one set of moments mu_0..mu_6 (Gauss-Legendre in
// ln(1+r/r_s) inside r_vir and ln r outside, where the integrands are
// analytic), after which the pressure condition is a degree-6 polynomial in a
// solved by safeguarded Newton, and the energy residual is a few Horner sums.
//
// K2: one workgroup per halo, one lane per table node; each node is a
// sight-line integral evaluated by Gauss-Legendre in s with l = r_perp sinh s,
// which removes both the sqrt edge at r_perp and the central cusp.
#include <hip/hip_runtime.h>
#include <math.h>

#include "bp_device.hpp"
#include "bp_internal.hpp"
#include "bp_footprint.hpp"

namespace bp {

// Per-halo constants of the solve (astrophysical units).
struct HaloSolve {
    double c, mc, rv, rs, V2, rhos;
    double Mg;       // f_b M - M_*  (gas mass inside r_f)
    double Ps;       // surface pressure
    double Egi;      // initial gas energy
    double Einj;     // eps_DM |E_DM| + eps_* M_* c^2
    double phi_out0; // c^2 / ((1+c) m(c)):  phi_out(r) = phi_out0 - r_vir/r
    double cm;       // c / m(c):  phi_in(x) = cm (1 - ln(1+x)/x)
    double gfac;     // (Gamma-1)/Gamma
    int energy_sign;
};

__device__ inline double binom(int n, int k) {
    const double t[8][8] = {{1}, {1, 1}, {1, 2, 1}, {1, 3, 3, 1}, {1, 4, 6, 4, 1}, {1, 5, 10, 10, 5, 1},
                            {1, 6, 15, 20, 15, 6, 1}, {1, 7, 21, 35, 35, 21, 7, 1}};
    return t[n][k];
}

// Moments mu_k = int_0^{r_f} 4 pi r^2 phi(r)^k dr, k = 0..6, in pieces.
// Inner part (r < r_vir): x = r/r_s, integrated in s = ln(1+x) by Gauss-Legendre, accumulated
// into mu over [Xa, Xb].
template <int NG>
__device__ __attribute__((always_inline)) inline void inner_moments(const HaloSolve &H, const double *gx, const double *gw, double Xa, double Xb,
                                     double mu[7]) {
    const double fourpi = 4.0 * kPi;
    const double Sa = log1p(Xa), Sb = log1p(Xb), hs = 0.5 * (Sb - Sa);
    const double rs3 = H.rs * H.rs * H.rs;
    for (int j = 0; j < NG; ++j) {
        double x = expm1(Sa + hs * (gx[j] + 1.0));
        double ph = H.cm * nfw_phi_shape(x);
        double w = hs * gw[j] * fourpi * rs3 * x * x * (1.0 + x);
        double pk = 1.0;
        for (int k = 0; k < 7; ++k) { mu[k] += w * pk; pk *= ph; }
    }
}

// Outer shell r_vir < r < r_f = x_f r_vir (x_f > 1), where phi = A - r_vir/r, A = phi_out0, in closed
// form: with u = r/r_vir, int 4 pi r^2 (A - 1/u)^k dr = 4 pi r_vir^3 sum_j C(k,j) A^(k-j) (-1)^j L_j,
// L_j = int_1^{x_f} u^(2-j) du, each written with d = x_f - 1 (exact) so nothing cancels.
__device__ inline void outer_moments(const HaloSolve &H, double xf, double mu[7]) {
    const double d = xf - 1.0, q = xf * xf + xf + 1.0, ix = 1.0 / xf;
    double L[7];
    L[0] = d * q / 3.0;                    // (x^3 - 1)/3
    L[1] = 0.5 * d * (xf + 1.0);           // (x^2 - 1)/2
    L[2] = d;                              // x - 1
    L[3] = log1p(d);                       // ln x
    L[4] = d * ix;                         // 1 - 1/x
    L[5] = 0.5 * d * (xf + 1.0) * ix * ix; // (1 - 1/x^2)/2
    L[6] = d * q * ix * ix * ix / 3.0;     // (1 - 1/x^3)/3
    const double c0 = 4.0 * kPi * H.rv * H.rv * H.rv, A = H.phi_out0;
    double Ap[7];
    Ap[0] = 1.0;
    for (int k = 1; k < 7; ++k) Ap[k] = Ap[k - 1] * A;
    for (int k = 0; k < 7; ++k) {
        double t = 0.0;
        for (int j = 0; j <= k; ++j) {
            double term = binom(k, j) * Ap[k - j] * L[j];
            t += (j & 1) ? -term : term;
        }
        mu[k] += c0 * t;
    }
}

__device__ inline double phi_at(const HaloSolve &H, double xf) {
    return xf > 1.0 ? H.phi_out0 - 1.0 / xf : H.cm * nfw_phi_shape(xf * H.c);
}

// I_n(a) = int 4 pi r^2 (1 - a phi)^n dr from the moments; J(a) = int 4 pi r^2 phi (1-a phi)^5 dr.
__device__ inline double poly_I(const double mu[7], int n, double a) {
    double s = 0.0, ak = 1.0;
    for (int k = 0; k <= n; ++k) { s += binom(n, k) * ak * mu[k]; ak *= -a; }
    return s;
}
__device__ inline double poly_J5(const double mu[7], double a) {
    double s = 0.0, ak = 1.0;
    for (int k = 0; k <= 5; ++k) { s += binom(5, k) * ak * mu[k + 1]; ak *= -a; }
    return s;
}

// Pressure condition for given moments: F(a) = gfac Mg V2 (1 - a phif)^6 - Ps a I5(a) = 0
// on (0, 1/phif).  F is a degree-6 polynomial with F(0) > 0 > F(1/phif); the
// root is unique on this interval for the model's parameter range.
__device__ double solve_a(const HaloSolve &H, const double mu[7], double phif, double a_guess) {
    double C0 = H.gfac * H.Mg * H.V2;
    // coefficients of F in powers of a
    double f[7];
    for (int k = 0; k < 7; ++k) {
        double t = C0 * binom(6, k);
        for (int q = 0; q < k; ++q) t *= -phif;
        f[k] = t;
    }
    for (int k = 0; k <= 5; ++k) {  // - Ps a sum C(5,k)(-a)^k mu_k
        double t = -H.Ps * binom(5, k) * mu[k];
        if (k & 1) t = -t;
        f[k + 1] += t;
    }
    double lo = 0.0, hi = 1.0 / phif;
    double a = (a_guess > lo && a_guess < hi) ? a_guess : 0.5 * hi;
    for (int it = 0; it < 100; ++it) {
        double F = f[6], dF = 0.0;
        for (int k = 5; k >= 0; --k) { dF = dF * a + F; F = F * a + f[k]; }
        if (F > 0) lo = a; else hi = a;
        double an = a - F / dF;
        const bool newton = an > lo && an < hi;
        if (!newton) an = 0.5 * (lo + hi);
        // a Newton step below 1e-9 relative leaves an error of order its square (the root is simple)
        const bool conv = newton ? fabs(an - a) <= 1e-9 * an : hi - lo <= 1e-15 * hi;
        a = an;
        if (conv) break;
    }
    return a;
}

struct Trial { double res, a, rho0, P0; };

// Energy residual (Sec. 2.2) at trial x_f from the moments of [0, r_f]; also returns a, rho0, P0.
__device__ Trial energy_trial(const HaloSolve &H, const double mu[7], double xf, double a_guess) {
    const double phif = phi_at(H, xf);
    Trial T;
    T.a = solve_a(H, mu, phif, a_guess);
    double I5 = poly_I(mu, 5, T.a), I6 = poly_I(mu, 6, T.a), J5 = poly_J5(mu, T.a);
    T.rho0 = H.Mg / I5;
    T.P0 = H.gfac * T.rho0 * H.V2 / T.a;
    double Phi0 = -H.V2 * H.phi_out0;
    double Egf = 1.5 * T.P0 * I6 + T.rho0 * (Phi0 * I5 + H.V2 * J5);
    double rf = xf * H.rv;
    double dEp = 4.0 * kPi / 3.0 * (H.rv * H.rv * H.rv - rf * rf * rf) * H.Ps;
    double res = (H.energy_sign == 0) ? Egf - (H.Egi + H.Einj + dEp) : H.Egi - (Egf + H.Einj + dEp);
    T.res = res / fabs(H.Egi);
    return T;
}

// Jeans integral I(x): closed form for x <= 2, else quadrature in s = ln(t/x)
// (the closed form cancels badly at large x).
__device__ double jeans_I_dev(double x, const GaussRules &G) {
    if (x <= 2.0) return jeans_I(x);
    const double smax = 12.0;  // integrand ~ s e^{-4s}
    double acc = 0.0;
    for (int j = 0; j < 24; ++j) {
        double s = 0.5 * smax * (G.x24[j] + 1.0);
        double t = x * exp(s);
        acc += G.w24[j] * nfw_m(t) * exp(-2.0 * s) / ((1.0 + t) * (1.0 + t));
    }
    return 0.5 * smax * acc / (x * x);
}

// Closed-form initial energy of matter in [x_lo, c] (without f_b): kinetic part
// by parts with the Jeans equation, potential part from elementary antiderivatives.
// Ic = jeans_I_dev(c), shared by the callers.
__device__ double energy_closed(double c, double mc, double A, double xlo, double Ic, const GaussRules &G) {
    double kin_b = c * c * c * Ic - (xlo > 0 ? xlo * xlo * xlo * jeans_I_dev(xlo, G) : 0.0);
    double K = 0.5 * A * (kin_b + kin_prim(c) - kin_prim(xlo));
    auto wprim = [&](double x) { return -log1p(x) / (1.0 + x) - 1.0 / (1.0 + x) - nfw_m(x) / (1.0 + c); };
    double W = -A * (wprim(c) - wprim(xlo));
    return K + W;
}

// Comoving-distance and optical-depth integrands on [0, z] by 24-point GL.
__device__ void distances(const bp_params &P, const GaussRules &G, double z, double *chi, double *tauint) {
    double a1 = 0.0, a2 = 0.0;
    for (int j = 0; j < 24; ++j) {
        double zz = 0.5 * z * (G.x24[j] + 1.0);
        double zp = 1.0 + zz;
        double E = sqrt(P.Omega_m * zp * zp * zp + 1.0 - P.Omega_m);
        a1 += G.w24[j] / E;
        a2 += G.w24[j] * zp * zp / E;
    }
    *chi = 0.5 * z * a1;     // in units of c/H0
    *tauint = 0.5 * z * a2;
}

// Brent's method (bisection / secant / inverse quadratic interpolation) for the energy residual on a
// bracket [a, b] with f(a) f(b) < 0, stopping at |b - c| <= 2 eps |b| + xtol; `trial(x, a_guess)`
// evaluates the residual at x (aguess carries the slope a from one trial to the next).  Returns b.
template <class F>
__device__ double brent_xf(F &&trial, double a, double b, double fa, double fbv, double xtol, double &aguess2) {
    double cc = a, fc = fa, d = b - a, e = d;
    for (int it = 0; it < 200; ++it) {
        if ((fbv > 0 && fc > 0) || (fbv < 0 && fc < 0)) { cc = a; fc = fa; d = b - a; e = d; }
        if (fabs(fc) < fabs(fbv)) { a = b; b = cc; cc = a; fa = fbv; fbv = fc; fc = fa; }
        double tol = 2.0 * 2.220446049250313e-16 * fabs(b) + 0.5 * xtol;
        double m = 0.5 * (cc - b);
        if (fabs(m) <= tol || fbv == 0.0) break;
        if (fabs(e) >= tol && fabs(fa) > fabs(fbv)) {
            double s = fbv / fa, p, q;
            if (a == cc) { p = 2.0 * m * s; q = 1.0 - s; }
            else {
                double qq = fa / fc, r = fbv / fc;
                p = s * (2.0 * m * qq * (qq - r) - (b - a) * (r - 1.0));
                q = (qq - 1.0) * (r - 1.0) * (s - 1.0);
            }
            if (p > 0) q = -q; else p = -p;
            if (2.0 * p < fmin(3.0 * m * q - fabs(tol * q), fabs(e * q))) { e = d; d = p / q; }
            else { d = m; e = m; }
        } else { d = m; e = m; }
        a = b; fa = fbv;
        b += (fabs(d) > tol) ? d : (m > 0 ? tol : -tol);
        Trial T = trial(b, aguess2);
        aguess2 = T.a;
        fbv = T.res;
    }
    return b;
}

#define NSCAN 47
// scan grid of the gas boundary x_f = r_f / r_vir: NSCAN points uniform on [0.4, 5]
__device__ inline double scan_x(int k) { return 0.4 + (5.0 - 0.4) * k / (NSCAN - 1); }

enum { kSolveScan = 0, kSolveStructure = 1, kSolveSeeded = 2 };

// Two waves per SIMD (at most 256 VGPRs, a few spilled): with one lane per halo the launch is only a
// few waves deep per SIMD, and at the unconstrained 262 VGPRs a single resident wave leaves every
// FP64 latency exposed (2.47 ms against 1.81 ms for 5e5 halos; three waves spill 110 VGPRs, 1.97 ms).
//   kSolveScan:      the exact solve (first sign change of the energy residual on the scan, then Brent);
//   kSolveStructure: the halo structure only (the surrogate's domain test; no boundary conditions);
//   kSolveSeeded:    the exact solve's root, found from the surrogate network's estimate of ln x_f
//                    (output 2 BP_MLP_NQ of yseed, standardised by ymean / ysd) instead of the scan:
//                    a bracket is widened from the estimate, then Brent to the same tolerance.  Halos
//                    outside the network's training domain get the structure and BP_S_OUT_OF_DOMAIN.
template <int kMode>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
k_icm_solve(bp_params P, GaussRules G, int64_t n, const double *__restrict__ Min, const double *__restrict__ cin,
            const double *__restrict__ zin, const float *__restrict__ yseed, const float *__restrict__ ymean,
            const float *__restrict__ ysd, double *__restrict__ sol, int32_t *__restrict__ status) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double M = Min[i], c = cin[i], z = zin[i];
    auto S = [&](int f) -> double & { return sol[(int64_t)f * n + i]; };
    for (int f = 0; f < BP_SOL_NFIELDS; ++f) S(f) = 0.0;
    S(BP_SOL_M) = M; S(BP_SOL_C) = c; S(BP_SOL_Z) = z;
    if (!(M > 0.0) || !(c > 0.0) || !(z >= 0.0) || !isfinite(M) || !isfinite(c) || !isfinite(z)) {
        status[i] = BP_S_BAD_INPUT;
        return;
    }
    int st = 0;
    const double h = P.h;
    // --- structure (Sec. 2.1) ---
    double zp = 1.0 + z, zp3 = zp * zp * zp;
    double E2 = P.Omega_m * zp3 + 1.0 - P.Omega_m;
    // rho_crit today in (Msun/h)/(Mpc/h)^3: 3 (100 km/s/Mpc)^2 / (8 pi G)
    double rho_c = 3.0 * 1e4 / (8.0 * kPi * kGastro) * E2;
    double xbn = P.Omega_m * zp3 / E2 - 1.0;
    double Dvir = 18.0 * kPi * kPi + 82.0 * xbn - 39.0 * xbn * xbn;
    double rv = cbrt(3.0 * M / (4.0 * kPi * Dvir * rho_c));
    double rs = rv / c, mc = nfw_m(c);
    double rhos = M / (4.0 * kPi * rs * rs * rs * mc);
    S(BP_SOL_RVIR) = rv; S(BP_SOL_RS) = rs; S(BP_SOL_RHOS) = rhos;

    // --- r500: ln(3 rho_s m(x)/x^3) = ln(500 rho_c), safeguarded Newton in ln x ---
    double target = log(500.0 * rho_c / (3.0 * rhos));
    double llo = log(c) - 30.0, lhi = log(c), lx = log(c) - 1.0;
    for (int it = 0; it < 200; ++it) {
        double x = exp(lx), m = nfw_m(x);
        double g = log(m) - 3.0 * lx - target;      // decreasing in ln x
        if (g > 0) llo = lx; else lhi = lx;
        double dg = x * nfw_dm(x) / m - 3.0;
        double ln_new = lx - g / dg;
        if (!(ln_new > llo && ln_new < lhi)) ln_new = 0.5 * (llo + lhi);
        if (fabs(ln_new - lx) < 1e-15 || lhi - llo < 1e-15) { lx = ln_new; break; }
        lx = ln_new;
    }
    double x500 = exp(lx);
    double r500 = x500 * rs, M500 = 4.0 * kPi * rhos * rs * rs * rs * nfw_m(x500);
    S(BP_SOL_R500) = r500; S(BP_SOL_M500) = M500;
    if (kMode != kSolveScan) {
        // the surrogate's training domain (log10 M, c, z)
        const double lm = log10(M);
        const bool in = lm >= 12.5 && lm <= 15.5 && c >= 2.0 && c <= 15.0 && z >= 0.05 && z <= 3.0;
        if (kMode == kSolveStructure || !in) {
            // the surrogate replaces everything from here to the tables; keep the exact geometry
            double chi_u, tau_u;
            distances(P, G, z, &chi_u, &tau_u);
            double cH = kCkms / 100.0, chi = cH * chi_u;
            S(BP_SOL_CHI) = chi;
            S(BP_SOL_DA) = chi / zp;
            double H0 = 100.0 * h * 1e5 / kMpc;
            double rho_cr0 = 3.0 * H0 * H0 / (8.0 * kPi * kG);
            double ne_bar = P.Omega_b * rho_cr0 / (2.0 / (1.0 + P.X_H) * kMp);
            S(BP_SOL_TAU) = kSigmaT * ne_bar * (kC / H0) * tau_u;
            double fmax = pow(4.0, -P.n_nt) / P.alpha_nt;
            S(BP_SOL_FNT) = fmin(pow(zp, P.beta_nt), (fmax - 1.0) * tanh(P.beta_nt * z) + 1.0);
            // surface pressure (the surrogate predicts the central pressure relative to it)
            const double fb0 = P.Omega_b / P.Omega_m;
            const double u_len0 = kMpc / h, u_mass0 = kMsun / h;
            S(BP_SOL_PS) = fb0 * 4.0 * kPi * kGastro * rhos * rhos * rs * rs * jeans_I_dev(c, G) * u_mass0 /
                           (u_len0 * u_len0 * u_len0) * 1e10;
            status[i] = in ? 0 : BP_S_OUT_OF_DOMAIN;
            return;
        }
    }

    // --- stars (Sec. 2.2); the 3e14 Msun pivot is in Msun ---
    double fb = P.Omega_b / P.Omega_m;
    double Fs = P.f_star * pow(M500 / h / 3e14, -P.S_star);
    double Mstar = Fs * M;
    S(BP_SOL_MSTAR) = Mstar;
    double ratio = Mstar / (fb * M);
    if (!(ratio < 1.0)) { status[i] = BP_S_NO_STAR_ROOT; return; }
    double mt = ratio * mc;
    double xlo = 0.0, xhi = c, xs = (mt < 1e-3) ? sqrt(2.0 * mt) : 0.5 * c;
    for (int it = 0; it < 200; ++it) {
        double g = nfw_m(xs) - mt;  // increasing
        if (g < 0) xlo = xs; else xhi = xs;
        double xn = xs - g / nfw_dm(xs);
        if (!(xn > xlo && xn < xhi)) xn = 0.5 * (xlo + xhi);
        if (fabs(xn - xs) <= 1e-15 * xn || xhi - xlo <= 1e-15 * xhi) { xs = xn; break; }
        xs = xn;
    }
    S(BP_SOL_XSTAR) = xs;

    // --- energies and surface pressure ---
    HaloSolve H;
    H.c = c; H.mc = mc; H.rv = rv; H.rs = rs; H.rhos = rhos;
    H.V2 = kGastro * M / rv;
    H.Mg = fb * M - Mstar;
    double A = kGastro * (M / mc) * (M / mc) / rs;  // G M0^2 / r_s
    const double Ic = jeans_I_dev(c, G);
    H.Ps = fb * 4.0 * kPi * kGastro * rhos * rhos * rs * rs * Ic;
    H.Egi = fb * energy_closed(c, mc, A, xs, Ic, G);
    double EDM = energy_closed(c, mc, A, 0.0, Ic, G);
    H.Einj = P.eps_DM * fabs(EDM) + P.eps_star * Mstar * kCkms * kCkms;
    H.phi_out0 = c * c / ((1.0 + c) * mc);
    H.cm = c / mc;
    H.gfac = (P.Gamma - 1.0) / P.Gamma;
    H.energy_sign = P.energy_sign;
    // unit conversions to CGS
    const double u_len = kMpc / h, u_mass = kMsun / h;
    const double u_rho = u_mass / (u_len * u_len * u_len);
    const double u_P = u_rho * 1e10;
    S(BP_SOL_PS) = H.Ps * u_P;
    S(BP_SOL_EGI) = H.Egi * u_mass * 1e10;

    double xf;
    Trial T;
    if (kMode == kSolveScan) {
        // --- scan x_f, then Brent on the first sign change ---
        // Moments of [0, r_f]: the inner part is carried along the increasing scan points up to
        // x_f = 1 (GL16 on the first piece, GL8 on each step), frozen at r_vir beyond, where the
        // outer shell has a closed form.  A Brent trial starts from the moments at its bracket's
        // lower end.
        double mu_cur[7] = {0, 0, 0, 0, 0, 0, 0}, x_cur = 0.4;
        inner_moments<16>(H, G.x16, G.w16, 0.0, 0.4 * c, mu_cur);
        double mu_vir[7];
        bool have_vir = false;
        auto moments_at = [&](const double base[7], double xbase, double xf, double mu[7]) {
            if (xf <= 1.0) {
                for (int k = 0; k < 7; ++k) mu[k] = base[k];
                if (xf > xbase) inner_moments<8>(H, G.x8, G.w8, xbase * c, xf * c, mu);
            } else {
                if (!have_vir) {
                    for (int k = 0; k < 7; ++k) mu_vir[k] = mu_cur[k];
                    if (x_cur < 1.0) inner_moments<8>(H, G.x8, G.w8, x_cur * c, c, mu_vir);
                    have_vir = true;
                }
                for (int k = 0; k < 7; ++k) mu[k] = mu_vir[k];
                outer_moments(H, xf, mu);
            }
        };
        double xprev = 0.0, rprev = 0.0, aprev = 0.0;
        double bx0 = 0.0, bx1 = 0.0, br0 = 0.0, br1 = 0.0, ba = 0.0;
        double mu_prev[7] = {0, 0, 0, 0, 0, 0, 0}, mu_b[7] = {0, 0, 0, 0, 0, 0, 0};
        int nchg = 0;
        double aguess = 0.0;
        for (int k = 0; k < NSCAN; ++k) {
            double xf = scan_x(k);
            double mu[7];
            if (xf <= 1.0) {
                moments_at(mu_cur, x_cur, xf, mu);
                for (int q = 0; q < 7; ++q) mu_cur[q] = mu[q];
                x_cur = xf;
            } else {
                moments_at(mu_cur, x_cur, xf, mu);
            }
            Trial T = energy_trial(H, mu, xf, aguess);
            // the next point starts from the linear extrapolation of a along the uniform scan
            aguess = k > 0 ? 2.0 * T.a - aprev : T.a;
            if (!isfinite(T.res)) { st |= BP_S_NONFINITE; break; }
            if (k > 0 && ((rprev < 0) != (T.res < 0))) {
                if (nchg == 0) {
                    bx0 = xprev; bx1 = xf; br0 = rprev; br1 = T.res; ba = aprev;
                    for (int q = 0; q < 7; ++q) mu_b[q] = mu_prev[q];
                }
                ++nchg;
            }
            xprev = xf; rprev = T.res; aprev = T.a;
            for (int q = 0; q < 7; ++q) mu_prev[q] = mu[q];
        }
        if (!st && nchg == 0) st |= BP_S_NO_BRACKET;
        if (st) { status[i] = st; return; }
        if (nchg > 1) st |= BP_S_MULTI_ROOT;
        auto trial_at = [&](double x, double ag) {
            double mu[7];
            moments_at(mu_b, bx0, x, mu);
            return energy_trial(H, mu, x, ag);
        };
        double xtol = 1e-13 * bx0, aguess2 = ba;
        xf = brent_xf(trial_at, bx0, bx1, br0, br1, xtol, aguess2);
        T = trial_at(xf, aguess2);
    } else {
        // --- seeded: the network's x_f, a bracket widened from it, then Brent ---
        // Each trial's moments are built exactly as the scan builds them (GL16 on [0, 0.4 c], one GL8
        // step per scan interval, GL8 from the last grid point below x_f), so the root agrees with the
        // scan's to the Brent tolerance.
        double mu_g[7] = {0, 0, 0, 0, 0, 0, 0}, mu_v[7];
        int kg_have = -1;
        bool have_v = false;
        auto grid_to = [&](int kg) __attribute__((always_inline)) {   // inner moments of [0, scan_x(kg)], kg <= the last point <= 1
            if (kg_have < 0 || kg < kg_have) {
                for (int q = 0; q < 7; ++q) mu_g[q] = 0.0;
                inner_moments<16>(H, G.x16, G.w16, 0.0, 0.4 * c, mu_g);
                kg_have = 0;
            }
            for (; kg_have < kg; ++kg_have)
                inner_moments<8>(H, G.x8, G.w8, scan_x(kg_have) * c, scan_x(kg_have + 1) * c, mu_g);
        };
        int kv = 0;                         // the last scan point at or below r_vir
        while (kv + 1 < NSCAN && scan_x(kv + 1) <= 1.0) ++kv;
        auto trial_s = [&](double x, double ag) __attribute__((always_inline)) {
            double mu[7];
            if (x <= 1.0) {
                int kg = 0;
                while (kg < kv && scan_x(kg + 1) <= x) ++kg;
                grid_to(kg);
                for (int q = 0; q < 7; ++q) mu[q] = mu_g[q];
                if (x > scan_x(kg)) inner_moments<8>(H, G.x8, G.w8, scan_x(kg) * c, x * c, mu);
            } else {
                if (!have_v) {
                    grid_to(kv);
                    for (int q = 0; q < 7; ++q) mu_v[q] = mu_g[q];
                    if (scan_x(kv) < 1.0) inner_moments<8>(H, G.x8, G.w8, scan_x(kv) * c, c, mu_v);
                    have_v = true;
                }
                for (int q = 0; q < 7; ++q) mu[q] = mu_v[q];
                outer_moments(H, x, mu);
            }
            return energy_trial(H, mu, x, ag);
        };
        const int c0 = 2 * BP_MLP_NQ;
        const double xg = exp((double)(yseed[i * BP_MLP_OUT + c0] * ysd[c0] + ymean[c0]));
        const double xs_lo = scan_x(0), xs_hi = scan_x(NSCAN - 1);
        double xa = isfinite(xg) ? fmin(fmax(xg, xs_lo), xs_hi) : 1.5;
        Trial Ta = trial_s(xa, 0.0);
        double fa = Ta.res;
        // second point 0.2% away (the network's x_f is typically within 1e-3); then secant steps that
        // overshoot by half until the residual changes sign (at most 8)
        double xb = xa * 1.002 <= xs_hi ? xa * 1.002 : xa * 0.998;
        Trial Tb = trial_s(xb, Ta.a);
        double fbv = Tb.res, agb = Tb.a;
        bool ok = isfinite(fa) && isfinite(fbv);
        for (int widen = 0; ok && ((fa < 0) == (fbv < 0)); ++widen) {
            const double slope = (fbv - fa) / (xb - xa), xsec = xb - fbv / slope;
            double xn = (isfinite(xsec) && slope != 0.0) ? xb + 1.5 * (xsec - xb) : xb + 2.0 * (xb - xa);
            xn = fmin(fmax(xn, xs_lo), xs_hi);
            if (widen >= 8 || xn == xb) { ok = false; break; }
            Trial Tn = trial_s(xn, agb);
            xa = xb; fa = fbv;
            xb = xn; fbv = Tn.res; agb = Tn.a;
            ok = isfinite(fbv);
        }
        if (!ok) {
            st |= isfinite(fa) && isfinite(fbv) ? BP_S_NO_BRACKET : BP_S_NONFINITE;
            status[i] = st;
            return;
        }
        double aguess2 = agb;
        xf = brent_xf(trial_s, xb, xa, fbv, fa, 1e-13 * fmin(xa, xb), aguess2);
        T = trial_s(xf, aguess2);
    }
    S(BP_SOL_A) = T.a;
    S(BP_SOL_XF) = xf;
    S(BP_SOL_RF) = xf * rv;
    S(BP_SOL_RHO0) = T.rho0 * u_rho;
    S(BP_SOL_P0) = T.P0 * u_P;
    S(BP_SOL_RES_E) = T.res;

    // --- distances, optical depth, non-thermal amplitude ---
    double chi_u, tau_u;
    distances(P, G, z, &chi_u, &tau_u);
    double cH = kCkms / 100.0;  // c/H0 in Mpc/h
    double chi = cH * chi_u;
    S(BP_SOL_CHI) = chi;
    S(BP_SOL_DA) = chi / zp;
    double H0 = 100.0 * h * 1e5 / kMpc;
    double rho_cr0 = 3.0 * H0 * H0 / (8.0 * kPi * kG);
    double ne_bar = P.Omega_b * rho_cr0 / (2.0 / (1.0 + P.X_H) * kMp);
    S(BP_SOL_TAU) = kSigmaT * ne_bar * (kC / H0) * tau_u;
    double fmax = pow(4.0, -P.n_nt) / P.alpha_nt;
    double fz = fmin(pow(zp, P.beta_nt), (fmax - 1.0) * tanh(P.beta_nt * z) + 1.0);
    S(BP_SOL_FNT) = fz;
    S(BP_SOL_RT) = fmin(xf * rv, P.trunc_r500 * r500);
    if (!isfinite(T.rho0) || !isfinite(T.P0) || !isfinite(xf)) st |= BP_S_NONFINITE;
    status[i] = st;
}

// ---------------------------------------------------------------- tables --
// Electron pressure and density relative to their central values at radius r
// (analytic profile, no cut at r_f: the table edge nodes need the limit).
// Line-of-sight integrand in FP32: the radius, the NFW potential shape and the polytrope are
// formed from FP64-derived constants; FP32 rounding of theta = 1 - a phi enters P ~ theta^6 as
// ~2e-6 / theta relative, well inside the deposit tolerance, and the GL sums are kept in FP64.
struct Prof {
    float rv, inv_rs, rf, cm, phi_out0, a, inv_r500, ant_f, n_nt;
};
__device__ inline float hw_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ inline float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// NFW potential shape 1 - ln(1+x)/x in FP32 without cancellation.  Below x = 2, with
// s = x/(2+x) and t = s^2, ln(1+x) = 2 atanh(s) gives 1 - ln(1+x)/x = (x - 2 t B(t))/(2+x),
// B(t) = sum_k t^k/(2k+3), every term positive (t <= 1/4, truncated after t^9: < 5e-8).
// Above, ln(1+x)/x <= 0.55 and the hardware logarithm keeps ~2e-7.
__device__ inline float nfw_shape_f(float x) {
    if (x < 2.0f) {
        const float r = hw_rcp(2.0f + x);
        const float sx = x * r, t = sx * sx;
        float B = 1.0f / 21.0f;
        B = fmaf(t, B, 1.0f / 19.0f); B = fmaf(t, B, 1.0f / 17.0f); B = fmaf(t, B, 1.0f / 15.0f);
        B = fmaf(t, B, 1.0f / 13.0f); B = fmaf(t, B, 1.0f / 11.0f); B = fmaf(t, B, 1.0f / 9.0f);
        B = fmaf(t, B, 1.0f / 7.0f);  B = fmaf(t, B, 1.0f / 5.0f);  B = fmaf(t, B, 1.0f / 3.0f);
        return (x - 2.0f * t * B) * r;
    }
    return 1.0f - 0.693147180559945f * hw_log2(1.0f + x) * hw_rcp(x);
}

__device__ inline void prof_eval(const Prof &Q, float r, float *pe, float *ne) {
    const float ph = (r < Q.rv) ? Q.cm * nfw_shape_f(r * Q.inv_rs) : Q.phi_out0 - Q.rv * hw_rcp(r);
    const float th = fmaxf(1.0f - Q.a * ph, 0.0f);
    const float th2 = th * th, th5 = th2 * th2 * th;
    // non-thermal fraction R_nt = alpha f(z) (r/r500)^n_nt
    const float rnt = Q.ant_f * hw_exp2(Q.n_nt * hw_log2(r * Q.inv_r500));
    const float fth = (rnt < 1.0f) ? 1.0f - rnt : 0.0f;
    *pe = th5 * th * fth;
    *ne = th5;
}
__device__ inline float cosh_f(float s) {
    const float e = hw_exp2(1.44269504088896f * s);
    return 0.5f * (e + hw_rcp(e));
}

// Zone-A node geometry shared by every halo whose footprint reaches r_a (eta_lo = 0, the usual
// case): per node k, xi = acosh(r_a / r_perp), r_perp / r_a, u / r_a and xi / (u / r_a).  The grid
// end is the single-precision eta_top the deposit reads back, so nodes sit where it looks for them.
// Every launch writes the same values (a function of constants only).
__device__ double g_nodeA[BP_TAB_NA][4];

__global__ void __launch_bounds__(BP_TAB_NA) k_node_geom(double eta_hi) {
    const int k = threadIdx.x;
    const double eta = eta_hi * k / (BP_TAB_NA - 1);
    const double xi = expm1(eta);
    // cosh and tanh of xi from one expm1 (no cancellation for small xi)
    const double em = expm1(xi), e = 1.0 + em, q = e * e + 1.0;
    const double c1 = 2.0 * e / q, c2 = em * (2.0 + em) / q;
    g_nodeA[k][0] = xi;
    g_nodeA[k][1] = c1;
    g_nodeA[k][2] = c2;
    g_nodeA[k][3] = xi > 0.0 ? xi / c2 : 0.0;
}

// Per-halo grid ranges and central values (one lane per halo): the zone ranges in eta, omega and
// zeta, P_e0 and n_e0, and the profile-shape constants of the table integrals.  Written to meta,
// from which the table kernels and the deposits read them: computing the constants here, once per
// halo, keeps their FP64 logarithm and divisions out of every wavefront of the table kernels.
__global__ void __launch_bounds__(256) k_table_setup(bp_params P, GaussRules G, int64_t n,
                                                     const double *__restrict__ sol, const int32_t *__restrict__ status,
                                                     float *__restrict__ meta) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    auto S = [&](int f) { return sol[(int64_t)f * n + i]; };
    float m[BP_META_NFIELDS] = {};
    if (!(status[i] & ~BP_S_MULTI_ROOT)) {
        const double rv = S(BP_SOL_RVIR), rf = S(BP_SOL_RF), Rt = S(BP_SOL_RT);
        const double ra = fmin(rv, rf);
        // zone ranges; the innermost sight line r_perp = 1e-5 r_a has the same eta for every halo
        const double eta_lo = log1p(acosh(ra / fmin(Rt, ra)));
        const bool shell = rf > rv;
        const double D = shell ? rf * rf - rv * rv : 0.0;
        const double sD = sqrt(D);
        double om_lo = 0.0, om_hi = 0.0, ze_lo = 0.0, ze_hi = 0.0;
        if (shell) {
            double rtop = fmin(Rt, rv);
            om_lo = asinh(sqrt(fmax(rv * rv - rtop * rtop, 0.0)) / sD);
            om_hi = asinh(rv / sD);
        }
        if (Rt > rv) { ze_lo = acosh(rf / Rt); ze_hi = acosh(rf / rv); }
        const double X = P.X_H;
        m[BP_META_ETA_LO] = (float)eta_lo;
        m[BP_META_ETA_HI] = (float)G.eta_top;
        m[BP_META_OM_LO] = (float)om_lo;
        m[BP_META_OM_HI] = (float)om_hi;
        m[BP_META_ZE_LO] = (float)ze_lo;
        m[BP_META_ZE_HI] = (float)ze_hi;
        m[BP_META_PE0] = (float)((2.0 * X + 2.0) / (5.0 * X + 3.0) * S(BP_SOL_P0));
        m[BP_META_NE0] = (float)(S(BP_SOL_RHO0) / (2.0 / (1.0 + X) * kMp));
        const double c = S(BP_SOL_C), mc = nfw_m(c);
        m[BP_META_PR_RV] = (float)rv;
        m[BP_META_PR_INV_RS] = (float)(1.0 / S(BP_SOL_RS));
        m[BP_META_PR_RF] = (float)rf;
        m[BP_META_PR_CM] = (float)(c / mc);
        m[BP_META_PR_PHI_OUT0] = (float)(c * c / ((1.0 + c) * mc));
        m[BP_META_PR_A] = (float)S(BP_SOL_A);
        m[BP_META_PR_INV_R500] = (float)(1.0 / S(BP_SOL_R500));
        m[BP_META_PR_ANT_F] = (float)(P.alpha_nt * S(BP_SOL_FNT));
    }
    for (int f = 0; f < BP_META_NFIELDS; ++f) meta[(int64_t)f * n + i] = m[f];
}

// One block per halo, one table node per thread.  Node positions come from the single-precision
// grid ranges in meta (the values the deposits interpolate with).
// One table node (both quantities) of halo i.
__device__ inline void table_node(const GaussRules &G, int64_t n, const double *__restrict__ sol,
                                  const int32_t *__restrict__ status, const float *__restrict__ meta,
                                  float *__restrict__ tab, float n_nt, int64_t i, int node) {
    auto S = [&](int f) { return sol[(int64_t)f * n + i]; };
    auto Mt = [&](int f) { return (double)meta[(int64_t)f * n + i]; };
    float *tP = tab + (int64_t)i * BP_TAB_STRIDE;
    float *tN = tP + BP_TAB_ZONE;
    if (status[i] & ~BP_S_MULTI_ROOT) {
        tP[node] = 0.0f; tN[node] = 0.0f;
        return;
    }
    // per-halo constants (wave-uniform); the profile-shape ones come from meta
    const double rv = S(BP_SOL_RVIR), rf = S(BP_SOL_RF), Rt = S(BP_SOL_RT);
    auto Mf = [&](int f) { return meta[(int64_t)f * n + i]; };
    Prof Q;
    Q.rv = Mf(BP_META_PR_RV); Q.inv_rs = Mf(BP_META_PR_INV_RS); Q.rf = Mf(BP_META_PR_RF);
    Q.cm = Mf(BP_META_PR_CM); Q.phi_out0 = Mf(BP_META_PR_PHI_OUT0);
    Q.a = Mf(BP_META_PR_A);
    Q.inv_r500 = Mf(BP_META_PR_INV_R500);
    Q.ant_f = Mf(BP_META_PR_ANT_F);
    Q.n_nt = n_nt;
    const double eta_lo = Mt(BP_META_ETA_LO), eta_hi = Mt(BP_META_ETA_HI);
    const double om_lo = Mt(BP_META_OM_LO), om_hi = Mt(BP_META_OM_HI);
    const double ze_lo = Mt(BP_META_ZE_LO), ze_hi = Mt(BP_META_ZE_HI);
    const double ra = fmin(rv, rf);
    const bool shell = rf > rv;
    const double D = shell ? rf * rf - rv * rv : 0.0;
    const double sD = sqrt(D);
    const bool zoneB = Rt > rv;

    double accP = 0.0, accN = 0.0;
    if (node < BP_TAB_NA) {
        // zone A: g_A = Y_A / (P_e0 u), Y_A = 2 int_0^xi P(r_perp cosh s) r_perp cosh s ds
        double xi, rp, f, th;             // th = tanh(xi) = u / r_a
        if (eta_lo == 0.0) {
            xi = g_nodeA[node][0];
            rp = ra * g_nodeA[node][1];
            th = g_nodeA[node][2];
            f = g_nodeA[node][3] / ra;   // 2 * (xi/2) / u
        } else {
            const double eta = eta_lo + (eta_hi - eta_lo) * node / (BP_TAB_NA - 1);
            xi = expm1(eta);
            // cosh and tanh of xi from one expm1 (no cancellation for small xi)
            const double em = expm1(xi), e = 1.0 + em, q = e * e + 1.0;
            rp = ra * (2.0 * e / q);
            th = em * (2.0 + em) / q;
            f = xi / (ra * th);
        }
        // Gauss-Legendre order by the length xi of the s-interval: over the benchmark's halo
        // population the worst relative quadrature error stays below 3e-8 (under the FP32
        // rounding of the integrand) with 6 points up to xi = 1.4, 8 up to 3.2, 10 up to 4.6,
        // 12 up to 6.0, 14 up to 7.6, 16 up to 9.0 and 20 beyond.  A wavefront runs the largest
        // order among its lanes anyway, so every lane takes that order: the rule is then the same
        // for the whole wavefront and its nodes and weights are scalar loads.
        int ngl = xi > 9.0 ? 20 : xi > 7.6 ? 16 : xi > 6.0 ? 14 : xi > 4.6 ? 12 : xi > 3.2 ? 10 : xi > 1.4 ? 8 : 6;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) ngl = max(ngl, __shfl_xor(ngl, o, 64));
        const int ng = __builtin_amdgcn_readfirstlane(ngl);
        if (xi < 1e-7) {  // limit r_perp -> r_a
            float pe, ne;
            prof_eval(Q, (float)ra, &pe, &ne);
            accP = 2.0 * pe; accN = 2.0 * ne;
        } else {
            const float *gu = ng == 20 ? G.u20 : ng == 16 ? G.u16 : ng == 14 ? G.u14 : ng == 12 ? G.u12
                              : ng == 10 ? G.u10 : ng == 8 ? G.u8 : G.u6;
            const double *gw = ng == 20 ? G.w20 : ng == 16 ? G.w16 : ng == 14 ? G.w14 : ng == 12 ? G.w12
                               : ng == 10 ? G.w10 : ng == 8 ? G.w8 : G.w6;
            const float rpf = (float)rp, raf = (float)ra, xif = (float)xi;
            for (int j = 0; j < ng; ++j) {
                float r = fminf(rpf * cosh_f(xif * gu[j]), raf);
                float pe, ne;
                prof_eval(Q, r, &pe, &ne);
                double w = gw[j] * (double)r;
                accP += w * pe; accN += w * ne;
            }
            accP *= f; accN *= f;
        }
        if (shell) {
            // Fold the shell r_vir < r < r_f that the same sight line crosses into the node, so the deposit
            // reads one table: g_T = (u g_A + (S - u) g_S) / S with S = sqrt(u^2 + D) and g_S interpolated
            // from zone S (cubic Lagrange in omega; written by the zone S/B kernel, which runs first).
            // FP32 with the forms the deposit used per pixel when it read zone S itself.  Y is smooth across
            // zone A; its only kink, where the line grazes r_vir, sits at the zone's end as (r_vir - r_perp)^(5/2).
            const float u = (float)(ra * th), Df = (float)D, isqD = (float)(1.0 / sD);
            const float S = __builtin_amdgcn_sqrtf(fmaf(u, u, Df));
            const double l2e = 1.4426950408889634;
            const float om2_lo = (float)(om_lo * l2e);
            const float om2_ih = om_hi > om_lo ? (float)((BP_TAB_NS - 1) / ((om_hi - om_lo) * l2e)) : 0.0f;
            const float om = __builtin_amdgcn_logf((u + S) * isqD);          // asinh(u / sqrt(D)) / ln 2
            float gSP, gSN;
            lagr4x2(tP, BP_TAB_ZONE, BP_TAB_NA, BP_TAB_NS, (om - om2_lo) * om2_ih, &gSP, &gSN);
            const float sh = Df * __builtin_amdgcn_rcpf(S + u);             // S - u without cancellation
            const float inv = __builtin_amdgcn_rcpf(S);
            accP = (double)((u * (float)accP + sh * gSP) * inv);
            accN = (double)((u * (float)accN + sh * gSN) * inv);
        }
    } else if (node < BP_TAB_NA + BP_TAB_NS) {
        // zone S: g_S = Y_S / (P_e0 (S - u_v)), Y_S over the shell r_vir < r < r_f
        if (shell) {
            int k = node - BP_TAB_NA;
            double om = om_lo + (om_hi - om_lo) * k / (BP_TAB_NS - 1);
            double uv = sD * sinh(om);
            double Sv = sqrt(uv * uv + D);
            double rp = sqrt(fmax(rv * rv - uv * uv, 0.0));
            rp = fmax(rp, 1e-7 * rv);
            double s0 = acosh(rv / rp), s1 = acosh(rf / rp);
            double hs = 0.5 * (s1 - s0);
            const float rpf = (float)rp;
            // 8 points: below 1e-11 relative on the shell segment
            for (int j = 0; j < 8; ++j) {
                float sj = (float)(s0 + hs * (G.x8[j] + 1.0));
                float r = fminf(fmaxf(rpf * cosh_f(sj), Q.rv), Q.rf);
                float pe, ne;
                prof_eval(Q, r, &pe, &ne);
                double w = G.w8[j] * (double)r;
                accP += w * pe; accN += w * ne;
            }
            double f = 2.0 * hs / (D / (Sv + uv));
            accP *= f; accN *= f;
        }
    } else {
        // zone B: g_B = Y_B / (P_e0 U), sight lines with r_perp >= r_vir
        if (zoneB) {
            int k = node - BP_TAB_NA - BP_TAB_NS;
            double ze = ze_lo + (ze_hi - ze_lo) * k / (BP_TAB_NB - 1);
            if (ze < 1e-7) {
                float pe, ne;
                prof_eval(Q, Q.rf, &pe, &ne);
                accP = 2.0 * pe; accN = 2.0 * ne;
            } else {
                const double em = expm1(ze), e = 1.0 + em, q = e * e + 1.0;
                const double rp = rf * (2.0 * e / q);
                const double U = rf * (em * (2.0 + em) / q);
                const float rpf = (float)rp, zef = (float)ze;
                // 8 points: below 1e-11 relative (zeta <= acosh(x_f))
                for (int j = 0; j < 8; ++j) {
                    float r = fmaxf(fminf(rpf * cosh_f(zef * G.u8[j]), Q.rf), Q.rv);
                    float pe, ne;
                    prof_eval(Q, r, &pe, &ne);
                    double w = G.w8[j] * (double)r;
                    accP += w * pe; accN += w * ne;
                }
                double f = ze / U;
                accP *= f; accN *= f;
            }
        }
    }
    tP[node] = (float)accP;
    tN[node] = (float)accN;
}

// Zone A: one 192-lane block per halo (three wavefronts, all running the same zone's code).
__global__ void __launch_bounds__(BP_TAB_NA) k_tables(GaussRules G, int64_t n, const double *__restrict__ sol,
                                                      const int32_t *__restrict__ status,
                                                      const float *__restrict__ meta, float *__restrict__ tab,
                                                      float n_nt) {
    table_node(G, n, sol, status, meta, tab, n_nt, blockIdx.x, threadIdx.x);
}

static_assert(BP_TAB_NS == 32 && BP_TAB_NB == 32, "k_tables_sb maps 32 nodes of each zone to half a wavefront");

// Zones S and B in their own launch: wavefront 0 of a block takes the 32 shell nodes of two halos,
// wavefront 1 their 32 outer nodes, so no wavefront runs both zones' code one after the other.
__global__ void __launch_bounds__(128) k_tables_sb(GaussRules G, int64_t n, const double *__restrict__ sol,
                                                   const int32_t *__restrict__ status,
                                                   const float *__restrict__ meta, float *__restrict__ tab,
                                                   float n_nt) {
    const int64_t i = 2 * (int64_t)blockIdx.x + ((threadIdx.x >> 5) & 1);
    if (i >= n) return;
    const int zone = threadIdx.x >> 6;                  // 0: S, 1: B
    table_node(G, n, sol, status, meta, tab, n_nt, i, BP_TAB_NA + zone * BP_TAB_NS + (threadIdx.x & 31));
}

// Projected profiles of solved halos at the surrogate's q nodes, by the exact tables' sight-line
// quadratures (Sec. 3.3): for r_perp = q_k R_t below r_a the part of the line inside r_a (Gauss-Legendre
// in s, l = r_perp sinh s, the order chosen by the length of the s-interval as for zone A) plus the
// shell r_vir < r < r_f (8 points); at or beyond r_a the line through the shell alone (8 points).  The
// integrand is the FP32 profile of the exact tables with the same FP32 constants.  Output per halo:
// qt[i][k] = Y_P / (P_e0 R_t E), qt[i][BP_MLP_NQ + k] = Y_n / (n_e0 R_t E), E = sqrt(1 - (q_k R_t / r_f)^2),
// q_k = (1 - cos(pi k / 63)) / 2 (the last node the limit from inside, q = 1 - 1e-6; the innermost sight
// line no closer than 1e-5 r_a, as in the zone tables); meta's PE0 and NE0 from the solved P0 and rho0.
// Layout of the work: a block takes 64 consecutive halos, lane = halo, and each of its four wavefronts
// takes every fourth node, so that the lanes of a wavefront share one node (and nearly one quadrature
// order) and read their halos' constants with coalesced loads from the SoA solution.  The values
// gather in LDS and leave as contiguous rows.
struct QNodes { double q[BP_MLP_NQ]; };
constexpr int kQH = 64;                     // halos per block
__global__ void __launch_bounds__(256) k_qtables_exact(bp_params P, GaussRules G, QNodes QN, int64_t n,
                                                       const double *__restrict__ sol,
                                                       const int32_t *__restrict__ status, int32_t ok_mask,
                                                       const uint32_t *__restrict__ skip, bool write_meta,
                                                       float *__restrict__ qt, float *__restrict__ meta) {
    __shared__ float tile[kQH][2 * BP_MLP_NQ + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * kQH, i = i0 + lane;
    // a halo marked in skip is left alone, its status not even read (another stream may be writing it)
    auto take = [&](int64_t h) { return !(skip && skip[h]) && (status[h] & ~ok_mask) == 0; };
    const bool live = i < n && take(i);
    // Every lane runs the node loop (a lane without a live halo computes on stand-in values and stores
    // nothing), so that the wavefront can agree on one Gauss-Legendre order per node: it runs the
    // largest order among its lanes anyway, and one order for all makes the rule's nodes and weights
    // scalar loads.
    {
        auto S = [&](int f) { return live ? sol[(int64_t)f * n + i] : 1.0; };
        const double rv = S(BP_SOL_RVIR), rf = live ? S(BP_SOL_RF) : 2.0, Rt = S(BP_SOL_RT), c = S(BP_SOL_C);
        const double mc = nfw_m(c);
        if (live && wave == 0 && write_meta) {
            const double X = P.X_H;
            meta[(int64_t)BP_META_PE0 * n + i] = (float)((2.0 * X + 2.0) / (5.0 * X + 3.0) * S(BP_SOL_P0));
            meta[(int64_t)BP_META_NE0 * n + i] = (float)(S(BP_SOL_RHO0) / (2.0 / (1.0 + X) * kMp));
            for (int f = 0; f < BP_META_PE0; ++f) meta[(int64_t)f * n + i] = 0.0f;
            for (int f = BP_META_PR_RV; f < BP_META_NFIELDS; ++f) meta[(int64_t)f * n + i] = 0.0f;
        }
        Prof Q;   // the constants k_table_setup stores for the zone tables, rounded the same way
        Q.rv = (float)rv; Q.inv_rs = (float)(1.0 / S(BP_SOL_RS)); Q.rf = (float)rf;
        Q.cm = (float)(c / mc); Q.phi_out0 = (float)(c * c / ((1.0 + c) * mc));
        Q.a = (float)S(BP_SOL_A); Q.inv_r500 = (float)(1.0 / S(BP_SOL_R500));
        Q.ant_f = (float)(P.alpha_nt * S(BP_SOL_FNT)); Q.n_nt = (float)P.n_nt;
        const double ra = fmin(rv, rf);
        const bool shell = rf > rv;           // then r_a = r_vir and the shell starts where zone A ends
        const float raf = (float)ra;
        for (int k = wave; k < BP_MLP_NQ; k += 4) {
            const double q = QN.q[k];
            const double rp = fmax(q * Rt, 1e-5 * ra);
            const float rpf = (float)rp;
            double accP = 0.0, accN = 0.0;
            const bool za = live && rp < ra;
            const double xi = za ? acosh(ra / rp) : 0.0;
            int ngl = xi > 9.0 ? 20 : xi > 7.6 ? 16 : xi > 6.0 ? 14 : xi > 4.6 ? 12 : xi > 3.2 ? 10 : xi > 1.4 ? 8 : 6;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) ngl = max(ngl, __shfl_xor(ngl, o, 64));
            const int ng = __builtin_amdgcn_readfirstlane(ngl);
            if (!live) continue;
            if (za) {
                const float *gu = ng == 20 ? G.u20 : ng == 16 ? G.u16 : ng == 14 ? G.u14 : ng == 12 ? G.u12
                                  : ng == 10 ? G.u10 : ng == 8 ? G.u8 : G.u6;
                const double *gw = ng == 20 ? G.w20 : ng == 16 ? G.w16 : ng == 14 ? G.w14 : ng == 12 ? G.w12
                                   : ng == 10 ? G.w10 : ng == 8 ? G.w8 : G.w6;
                const float xif = (float)xi;
                double sP = 0.0, sN = 0.0;
                for (int j = 0; j < ng; ++j) {
                    float r = fminf(rpf * cosh_f(xif * gu[j]), raf);
                    float pe, ne;
                    prof_eval(Q, r, &pe, &ne);
                    const double w = gw[j] * (double)r;
                    sP += w * pe; sN += w * ne;
                }
                accP = xi * sP; accN = xi * sN;
                if (shell) {   // the shell r_vir < r < r_f crossed by the same line: s from xi to acosh(r_f / r_perp)
                    const double hs = 0.5 * (acosh(rf / rp) - xi);
                    double tP = 0.0, tN = 0.0;
                    for (int j = 0; j < 8; ++j) {
                        float r = fminf(fmaxf(rpf * cosh_f((float)(xi + hs * (G.x8[j] + 1.0))), Q.rv), Q.rf);
                        float pe, ne;
                        prof_eval(Q, r, &pe, &ne);
                        const double w = G.w8[j] * (double)r;
                        tP += w * pe; tN += w * ne;
                    }
                    accP += 2.0 * hs * tP; accN += 2.0 * hs * tN;
                }
            } else if (rp < rf) {
                const double ze = acosh(rf / rp);
                const float zef = (float)ze;
                double sP = 0.0, sN = 0.0;
                for (int j = 0; j < 8; ++j) {
                    float r = fmaxf(fminf(rpf * cosh_f(zef * G.u8[j]), Q.rf), Q.rv);
                    float pe, ne;
                    prof_eval(Q, r, &pe, &ne);
                    const double w = G.w8[j] * (double)r;
                    sP += w * pe; sN += w * ne;
                }
                accP = ze * sP; accN = ze * sN;
            }
            const double x = q * Rt / rf;
            const double norm = 1.0 / (Rt * sqrt(fmax(1.0 - x * x, 0.0)));
            tile[lane][k] = (float)(accP * norm);
            tile[lane][BP_MLP_NQ + k] = (float)(accN * norm);
        }
    }
    __syncthreads();
    // rows of the live halos out, 2 BP_MLP_NQ consecutive floats each
    const int nh = (int)min((int64_t)kQH, n - i0);
    for (int e = threadIdx.x; e < nh * 2 * BP_MLP_NQ; e += 256) {
        const int h = e / (2 * BP_MLP_NQ), k = e - h * 2 * BP_MLP_NQ;
        if (take(i0 + h)) qt[(i0 + h) * 2 * BP_MLP_NQ + k] = tile[h][k];
    }
}

// ------------------------------------------------------- Gauss-Legendre --
// Nodes and weights of the n-point rule on [-1,1] by Newton iteration on P_n.
static void gauss_legendre(int n, double *x, double *w) {
    for (int i = 0; i < n; ++i) {
        double z = cos(kPi * (i + 0.75) / (n + 0.5)), pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) { double p3 = p2; p2 = p1; p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j; }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            double z1 = z;
            z = z1 - p1 / pp;
            if (fabs(z - z1) < 1e-16) break;
        }
        x[i] = -z;
        w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

const GaussRules &gauss_rules() {
    static GaussRules G;
    static bool init = false;
    if (!init) {
        gauss_legendre(16, G.x16, G.w16);
        gauss_legendre(24, G.x24, G.w24);
        gauss_legendre(12, G.x12, G.w12);
        gauss_legendre(8, G.x8, G.w8);
        gauss_legendre(20, G.x20, G.w20);
        for (int j = 0; j < 16; ++j) G.u16[j] = (float)(0.5 * (G.x16[j] + 1.0));
        for (int j = 0; j < 12; ++j) G.u12[j] = (float)(0.5 * (G.x12[j] + 1.0));
        for (int j = 0; j < 8; ++j) G.u8[j] = (float)(0.5 * (G.x8[j] + 1.0));
        for (int j = 0; j < 20; ++j) G.u20[j] = (float)(0.5 * (G.x20[j] + 1.0));
        double xt[14];
        gauss_legendre(6, xt, G.w6);
        for (int j = 0; j < 6; ++j) G.u6[j] = (float)(0.5 * (xt[j] + 1.0));
        gauss_legendre(10, xt, G.w10);
        for (int j = 0; j < 10; ++j) G.u10[j] = (float)(0.5 * (xt[j] + 1.0));
        gauss_legendre(14, xt, G.w14);
        for (int j = 0; j < 14; ++j) G.u14[j] = (float)(0.5 * (xt[j] + 1.0));
        G.eta_top = log1p(acosh(1e5));
        init = true;
    }
    return G;
}

}  // namespace bp

using namespace bp;

// The kernels are written for the paper's adiabatic index Gamma = 1.2 (Sec. 2.1, Table 1), i.e. the
// polytropic index n = 1/(Gamma - 1) = 5: the moment expansion of the gas-mass and pressure
// conditions (binomials of order 5 and 6), the table integrand theta^5 and theta^6 and the particle
// amplitudes use it as a constant.  Any other Gamma is an argument error, not a silent misfit.
int bp::check_params(const bp_params *p) {
    if (!p) return BP_E_ARG;
    if (!(p->Omega_m > 0 && p->Omega_m <= 1.0) || !(p->Omega_b > 0 && p->Omega_b < p->Omega_m) || !(p->h > 0) ||
        p->Gamma != 1.2 || !(p->alpha_nt > 0) || !(p->n_nt > 0) || !(p->trunc_r500 > 0) ||
        !(p->X_H > 0 && p->X_H <= 1) || (p->energy_sign != 0 && p->energy_sign != 1) ||
        !(p->field_gas_frac >= 0 && p->field_gas_frac <= 1) || !(p->field_T >= 0 && p->field_T < 1e12) ||
        !(p->eps_DM >= 0 && p->eps_DM < 1e3) || !(p->eps_star >= 0 && p->eps_star < 1e3) ||
        !(p->f_star >= 0 && p->f_star < 1e3) || !(p->S_star > -1e3 && p->S_star < 1e3) ||
        !(p->beta_nt > -1e3 && p->beta_nt < 1e3))
        return BP_E_ARG;
    return BP_OK;
}

extern "C" int bp_icm_solve(const bp_params *p, int64_t n, const double *M, const double *c, const double *z,
                            double *sol, int32_t *status, void *stream) {
    int e = check_params(p);
    if (e) return e;
    if (n < 0) return BP_E_ARG;
    if (n == 0) return BP_OK;
    if (!M || !c || !z || !sol || !status) return BP_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    int64_t blocks = (n + 63) / 64;
    if (blocks > 0x7fffffff) return BP_E_OVERFLOW;
    prof_begin(BP_PROF_ICM, s);
    hipLaunchKernelGGL(k_icm_solve<kSolveScan>, dim3((unsigned)blocks), dim3(64), 0, s, *p, gauss_rules(), n, M, c, z,
                       nullptr, nullptr, nullptr, sol, status);
    prof_end(BP_PROF_ICM, s);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

int bp::profile_tables_launch(const bp_params *p, int64_t n, const double *sol, const int32_t *status, float *tables,
                              float *meta, hipStream_t s, hipEvent_t meta_ready) {
    int e = check_params(p);
    if (e) return e;
    if (n < 0) return BP_E_ARG;
    if (n == 0) return BP_OK;
    if (!sol || !status || !tables || !meta) return BP_E_ARG;
    if (n > 0x7fffffff) return BP_E_OVERFLOW;
    const GaussRules G = gauss_rules();
    prof_begin(BP_PROF_TABLES, s);
    hipLaunchKernelGGL(k_node_geom, dim3(1), dim3(BP_TAB_NA), 0, s, (double)(float)G.eta_top);
    hipLaunchKernelGGL(k_table_setup, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, *p, G, n, sol, status, meta);
    if (meta_ready && hipEventRecord(meta_ready, s) != hipSuccess) return BP_E_HIP;
    // zones S and B first: zone A folds the shell part of each of its sight lines in from zone S
    hipLaunchKernelGGL(k_tables_sb, dim3((unsigned)((n + 1) / 2)), dim3(128), 0, s, G, n, sol, status, meta,
                       tables, (float)p->n_nt);
    hipLaunchKernelGGL(k_tables, dim3((unsigned)n), dim3(BP_TAB_NA), 0, s, G, n, sol, status, meta, tables,
                       (float)p->n_nt);
    prof_end(BP_PROF_TABLES, s);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

extern "C" int bp_profile_tables(const bp_params *p, int64_t n, const double *sol, const int32_t *status,
                                 float *tables, float *meta, void *stream) {
    return profile_tables_launch(p, n, sol, status, tables, meta, (hipStream_t)stream, nullptr);
}

extern "C" int bp_halo_structure(const bp_params *p, int64_t n, const double *M, const double *c, const double *z,
                                 double *sol, int32_t *status, void *stream) {
    int e = check_params(p);
    if (e) return e;
    if (n < 0) return BP_E_ARG;
    if (n == 0) return BP_OK;
    if (!M || !c || !z || !sol || !status) return BP_E_ARG;
    int64_t blocks = (n + 63) / 64;
    if (blocks > 0x7fffffff) return BP_E_OVERFLOW;
    hipLaunchKernelGGL(k_icm_solve<kSolveStructure>, dim3((unsigned)blocks), dim3(64), 0, (hipStream_t)stream, *p,
                       gauss_rules(), n, M, c, z, nullptr, nullptr, nullptr, sol, status);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

extern "C" int bp_surrogate_solve(const bp_params *p, int64_t n, const double *M, const double *c, const double *z,
                                  const float *y, const float *mean, const float *std, double *sol, int32_t *status,
                                  void *stream) {
    int e = check_params(p);
    if (e) return e;
    if (n < 0) return BP_E_ARG;
    if (n == 0) return BP_OK;
    if (!M || !c || !z || !y || !mean || !std || !sol || !status) return BP_E_ARG;
    int64_t blocks = (n + 63) / 64;
    if (blocks > 0x7fffffff) return BP_E_OVERFLOW;
    hipStream_t s = (hipStream_t)stream;
    prof_begin(BP_PROF_SURR_SOLVE, s);
    hipLaunchKernelGGL(k_icm_solve<kSolveSeeded>, dim3((unsigned)blocks), dim3(64), 0, s, *p, gauss_rules(), n, M, c,
                       z, y, mean, std, sol, status);
    prof_end(BP_PROF_SURR_SOLVE, s);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

int bp::qtables_exact(const bp_params *p, int64_t n, const double *sol, const int32_t *status, int32_t ok_mask,
                      float *qtables, float *meta, hipStream_t s, const uint32_t *skip, bool write_meta) {
    int e = check_params(p);
    if (e) return e;
    if (n < 0) return BP_E_ARG;
    if (n == 0) return BP_OK;
    if (!sol || !status || !qtables || !meta) return BP_E_ARG;
    if (n > ((int64_t)1 << 40)) return BP_E_OVERFLOW;
    QNodes QN;
    for (int k = 0; k < BP_MLP_NQ; ++k) QN.q[k] = 0.5 * (1.0 - cos(kPi * k / (BP_MLP_NQ - 1)));
    QN.q[BP_MLP_NQ - 1] = 1.0 - 1e-6;
    prof_begin(BP_PROF_SURR_APPLY, s);
    hipLaunchKernelGGL(k_qtables_exact, dim3((unsigned)((n + kQH - 1) / kQH)), dim3(256), 0, s, *p, gauss_rules(), QN, n,
                       sol, status, ok_mask, skip, write_meta, qtables, meta);
    prof_end(BP_PROF_SURR_APPLY, s);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

extern "C" int bp_surrogate_qtables_exact(const bp_params *p, int64_t n, const double *sol, const int32_t *status,
                                          float *qtables, float *meta, void *stream) {
    return qtables_exact(p, n, sol, status, 0, qtables, meta, (hipStream_t)stream);
}
