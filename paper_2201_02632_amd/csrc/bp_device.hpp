// Device-side helpers shared by the libbp kernels (gfx950).
//
// Physical constants: CODATA-2018 and IAU values (the paper prints none).
// Astrophysical working units on the device: masses Msun/h, lengths
// physical Mpc/h, velocities km/s; energies Msun/h (km/s)^2; pressures
// Msun/h (km/s)^2 / (Mpc/h)^3.  Conversion to CGS happens at the edges.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bp.h"

namespace bp {

// ---- constants (CGS) -------------------------------------------------------
constexpr double kSigmaT = 6.6524587321e-25;      // cm^2
constexpr double kMeC2 = 8.1871057769e-7;         // erg
constexpr double kC = 2.99792458e10;              // cm/s
constexpr double kMp = 1.67262192369e-24;         // g
constexpr double kG = 6.67430e-8;                 // cm^3 g^-1 s^-2
constexpr double kMsun = 1.988409870698051e33;    // g
constexpr double kMpc = 3.0856775814913673e24;    // cm
constexpr double kKB = 1.380649e-16;              // erg/K
constexpr double kPi = 3.141592653589793238462643;
constexpr double kCkms = kC * 1e-5;               // km/s
// G in Mpc (km/s)^2 / Msun; with masses in Msun/h and lengths in Mpc/h the h cancels in G M / r
constexpr double kGastro = kG * kMsun / (kMpc * 1e10);

// Gauss-Legendre rules passed by value in kernel arguments (nodes on [-1,1]).
struct GaussRules {
    double x16[16], w16[16];
    double x24[24], w24[24];
    double x12[12], w12[12];
    double x8[8], w8[8];
    double x20[20], w20[20];
    float u16[16], u12[12], u8[8], u20[20];   // (x + 1) / 2 in FP32: nodes on [0, 1]
    double w6[6], w10[10], w14[14];           // further zone-A orders (weights; nodes only as u)
    float u6[6], u10[10], u14[14];
    double eta_top;                    // ln(1 + acosh(1e5)): zone-A grid end (r_perp = 1e-5 r_a)
};

// ---- NFW helpers ------------------------------------------------------------
// m(x) = ln(1+x) - x/(1+x); Taylor series below 1e-3 avoids the cancellation.
__host__ __device__ inline double nfw_m(double x) {
    if (x < 1e-3) {
        // x^2/2 - 2x^3/3 + 3x^4/4 - 4x^5/5 + 5x^6/6 - 6x^7/7
        double x2 = x * x;
        return x2 * (0.5 + x * (-2.0 / 3.0 + x * (0.75 + x * (-0.8 + x * (5.0 / 6.0 + x * (-6.0 / 7.0))))));
    }
    return log1p(x) - x / (1.0 + x);
}

// dm/dx = x / (1+x)^2
__host__ __device__ inline double nfw_dm(double x) { return x / ((1.0 + x) * (1.0 + x)); }

// 1 - ln(1+x)/x, the inner potential shape; series below 1e-3.
__host__ __device__ inline double nfw_phi_shape(double x) {
    if (x < 1e-3) return x * (0.5 + x * (-1.0 / 3.0 + x * (0.25 + x * (-0.2 + x * (1.0 / 6.0)))));
    return 1.0 - log1p(x) / x;
}

// Dilogarithm Li2(-x) for x >= 0 via the Bernoulli-number series
//   Li2(w) = sum_n B_n u^(n+1)/(n+1)!,  u = -ln(1-w),
// which converges for |u| < 2 pi; here u = -ln(1+x) with x <= 1 so |u| <= ln 2.
// Larger x use the inversion Li2(-x) = -pi^2/6 - ln^2(x)/2 - Li2(-1/x).
__host__ __device__ inline double li2_neg_small(double x) {
    // coefficients B_n/(n+1)! for n = 0,1,2,4,...,18
    const double u = -log1p(x);
    const double u2 = u * u;
    const double c[10] = {
        1.0 / 36.0,                             // B2/3!
        -1.0 / 30.0 / 120.0,                    // B4/5!
        1.0 / 42.0 / 5040.0,                    // B6/7!
        -1.0 / 30.0 / 362880.0,                 // B8/9!
        5.0 / 66.0 / 39916800.0,                // B10/11!
        -691.0 / 2730.0 / 6227020800.0,         // B12/13!
        7.0 / 6.0 / 1307674368000.0,            // B14/15!
        -3617.0 / 510.0 / 355687428096000.0,    // B16/17!
        43867.0 / 798.0 / 121645100408832000.0, // B18/19!
        0.0};
    // sum_{k} c_k u^(2k+3) + u - u^2/4
    double s = 0.0;
    for (int k = 8; k >= 0; --k) s = s * u2 + c[k];
    return u - 0.25 * u2 + s * u2 * u;
}
__host__ __device__ inline double li2_neg(double x) {
    if (x <= 1.0) return li2_neg_small(x);
    double l = log(x);
    return -kPi * kPi / 6.0 - 0.5 * l * l - li2_neg_small(1.0 / x);
}

// I(x) = int_x^inf m(t)/(t^3 (1+t)^2) dt in closed form (isotropic NFW Jeans
// integral, Lokas & Mamon form): sigma^2 = 4 pi G rho_s r_s^2 x (1+x)^2 I(x).
__host__ __device__ inline double jeans_I(double x) {
    double l1 = log1p(x), ix = 1.0 / x, ip = 1.0 / (1.0 + x);
    return 0.5 * (kPi * kPi - log(x) - ix - ip * ip - 6.0 * ip + (1.0 + ix * ix - 4.0 * ix - 2.0 * ip) * l1 +
                  3.0 * l1 * l1 + 6.0 * li2_neg(x));
}

// Energy antiderivatives used by the closed-form initial energy.
__host__ __device__ inline double kin_prim(double x) {
    double ip = 1.0 / (1.0 + x);
    return -log1p(x) * ip - 0.5 * ip * ip;
}

}  // namespace bp
