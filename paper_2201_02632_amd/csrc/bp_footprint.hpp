// Per-pixel evaluation of a halo's projected footprint from its zone tables
// (shared by the flat-sky and HEALPix deposits).
#pragma once

#include <hip/hip_runtime.h>

#include "bp_device.hpp"

namespace bp {

// Two tables (P at tab[base ..], n at tab[nofs + base ..]) sampled at the same position: cubic
// Lagrange through nodes i-1 .. i+2, with the weights written through a = f(f-1) and
// (f+1)(f-2) = a - 2.  tab is the halo's (wave-uniform) table pointer and the node index a 32-bit
// offset from it, so the loads take the scalar-base form.
__device__ inline void lagr4x2(const float *__restrict__ tab, int nofs, int base, int n, float s, float *vp,
                               float *vn) {
    // truncation instead of floor: the two differ only for s < 0, where the clamp gives 1 either way
    int i = (int)s;
    i = min(max(i, 1), n - 3);
    const float f = s - (float)i;
    const float fm1 = f - 1.0f;
    const float a = f * fm1;
    const float t = a * (-1.0f / 6.0f), u = (a - 2.0f) * 0.5f;
    const float w0 = t * (f - 2.0f);     // -f (f-1) (f-2) / 6
    const float w3 = -t * (f + 1.0f);    //  (f+1) f (f-1) / 6
    const float w1 = u * fm1;            //  (f+1) (f-1) (f-2) / 2
    const float w2 = -u * f;             // -(f+1) f (f-2) / 2
    const unsigned k = (unsigned)(base + i - 1);
    const float *p = tab + k, *q = tab + nofs + k;
    *vp = w0 * p[0] + w1 * p[1] + w2 * p[2] + w3 * p[3];
    *vn = w0 * q[0] + w1 * q[1] + w2 * q[2] + w3 * q[3];
}

// max(x, y) for y >= +0 and x not a NaN, as one integer max: non-negative floats order like their
// bit patterns, and a negative float (sign bit set) is below all of them.  fmaxf costs a second
// instruction here, which quiets a possible signalling NaN first.
__device__ inline float fmax_nn(float x, float y) {
    return __int_as_float(max(__float_as_int(x), __float_as_int(y)));
}

__device__ inline void kahan_add(float &s, float &c, float v) {
    float y = v - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Hardware transcendental approximations (about 1 ulp): the table coordinates they feed are
// smooth functions sampled at ~1e-2 spacing, so their rounding moves a pixel's value by
// well under 1e-6 relative.
__device__ inline float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline float hw_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Projected profile at squared impact parameter r2 (in the record's length
// unit), in units of the central electron pressure / density times that
// length.  u2 = r_a^2 - r2 and U2 = r_f^2 - r2 are passed in so the caller can
// form them without cancellation next to the footprint edge.
//   zone A (r < r_a):  Y = S g_T(eta),  eta = ln(1 + acosh(r_a / r)),  S = sqrt(u^2 + D),
//                      u = sqrt(r_a^2 - r^2), D = r_f^2 - r_vir^2 for a gas shell beyond r_vir (else 0):
//                      the table holds the whole line, the shell's part folded in
//   zone B (r >= r_a): Y = U g_B(zeta), zeta = acosh(r_f / r),        U = sqrt(r_f^2 - r^2)
// A and B share one interpolation with a per-lane table offset, so a wave that straddles r_a
// does not run both branches.  The grid coordinates are kept in log2 units (set_zone_grids), so
// each logarithm is one hardware log2 with no rescaling.
struct FootRec {
    float ra, rf, r2min, D, isqD, eta_lo, eta_ih, om_lo, om_ih, ze_lo, ze_ih;
    int flags;
};

// Zone grids of a table in log2 units: a coordinate c on [lo, hi] with N nodes becomes
// (c / ln 2 - lo / ln 2) * ((N - 1) ln 2 / (hi - lo)).
template <class Rec>
__host__ __device__ inline void set_zone_grids(Rec &r, float elo, float ehi, float olo, float ohi, float zlo, float zhi) {
    const double l2e = 1.4426950408889634;   // 1 / ln 2
    r.eta_lo = (float)((double)elo * l2e);
    r.eta_ih = (float)((BP_TAB_NA - 1) / (((double)ehi - (double)elo) * l2e));
    r.om_lo = (float)((double)olo * l2e);
    r.om_ih = (ohi > olo) ? (float)((BP_TAB_NS - 1) / (((double)ohi - (double)olo) * l2e)) : 0.0f;
    r.ze_lo = (float)((double)zlo * l2e);
    r.ze_ih = (zhi > zlo) ? (float)((BP_TAB_NB - 1) / (((double)zhi - (double)zlo) * l2e)) : 0.0f;
}

// The fields of a wave-uniform record, read once per (tile, halo) pair: readfirstlane is
// convergent, so the compiler keeps these reads outside the per-pixel branches.
__device__ inline float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
template <class Rec>
__device__ inline FootRec foot_uniform(const Rec &R) {
    FootRec F;
    F.ra = uni(R.ra); F.rf = uni(R.rf); F.r2min = uni(R.r2min); F.D = uni(R.D); F.isqD = uni(R.isqD);
    F.eta_lo = uni(R.eta_lo); F.eta_ih = uni(R.eta_ih); F.om_lo = uni(R.om_lo); F.om_ih = uni(R.om_ih);
    F.ze_lo = uni(R.ze_lo); F.ze_ih = uni(R.ze_ih);
    F.flags = __builtin_amdgcn_readfirstlane(R.flags);
    return F;
}

template <class Rec>
__device__ inline void footprint_value(const Rec &R, const float *__restrict__ tab, float r2, float u2, float U2,
                                       float *vp, float *vn) {
    const float kLn2 = 0.693147180559945f;
    const bool zA = u2 > 0.0f;
    const float w = hw_sqrt(fmax_nn(zA ? u2 : U2, 0.0f));                        // u or U
    // log2 of (r_{a,f} + w) / r = acosh(r_{a,f} / r) / ln 2
    const float L = __builtin_amdgcn_logf(((zA ? R.ra : R.rf) + w) * hw_rsq(fmax_nn(r2, R.r2min)));
    const float eta = __builtin_amdgcn_logf(fmaf(kLn2, fmax_nn(L, 0.0f), 1.0f));   // eta / ln 2
    const float sidx = zA ? (eta - R.eta_lo) * R.eta_ih : (L - R.ze_lo) * R.ze_ih;
    const int off = zA ? 0 : BP_TAB_NA + BP_TAB_NS;
    const int nn = zA ? BP_TAB_NA : BP_TAB_NB;
    float gp, gn;
    lagr4x2(tab, BP_TAB_ZONE, off, nn, sidx, &gp, &gn);
    // zone A holds the whole sight line, its shell part included: Y = S g_T with S = sqrt(u^2 + D)
    // (D = 0 without a shell, S = u); zone B: Y = U g_B
    const float e = zA ? hw_sqrt(fmaf(w, w, R.D)) : w;
    *vp = gp * e; *vn = gn * e;
}


// acos on [-1, 1] from the Hastings approximation of Abramowitz & Stegun 4.4.46 (absolute error
// below 2e-8 on [0, 1]): acos(x) = sqrt(1 - x) P(x) for x >= 0, pi - acos(-x) below.  Written for
// x = 1 - 2q, q in [0, 1], where 1 - x = 2q and 1 + x = 2 (1 - q) keep their digits.
__device__ inline float acos_1m2q(float q) {
    const bool hi = q > 0.5f;
    const float x = hi ? 2.0f * q - 1.0f : 1.0f - 2.0f * q;      // |1 - 2q|
    const float t = hi ? 2.0f * (1.0f - q) : 2.0f * q;           // 1 - |1 - 2q|
    float p = -0.0012624911f;
    p = fmaf(p, x, 0.0066700901f); p = fmaf(p, x, -0.0170881256f); p = fmaf(p, x, 0.0308918810f);
    p = fmaf(p, x, -0.0501743046f); p = fmaf(p, x, 0.0889789874f); p = fmaf(p, x, -0.2145988016f);
    p = fmaf(p, x, 1.5707963050f);
    const float a = hw_sqrt(t) * p;
    return hi ? 3.14159265358979f - a : a;
}

// Surrogate tables: 64 nodes per quantity at q_k = (1 - cos(pi k/63))/2, q = r_perp/R_t,
// interpolated in s = acos(1 - 2q)/pi.  R.eta_lo holds R_t and R.eta_ih 1/R_t (record units).
// Y = P_e0 R_t E G(q) with E = sqrt(1 - r_perp^2 / r_f^2) = sqrt(U2) / r_f.  The surrogate's own
// error (~1e-3) sets the precision here: hardware square roots and reciprocal.
template <class Rec>
__device__ inline void footprint_value_q(const Rec &R, const float *__restrict__ tab, float r2, float U2, float *vp,
                                         float *vn) {
    const float q = fminf(hw_sqrt(r2) * R.eta_ih, 1.0f);
    const float sidx = acos_1m2q(q) * (63.0f / 3.14159265358979f);
    float gp, gn;
    lagr4x2(tab, BP_MLP_NQ, 0, BP_MLP_NQ, sidx, &gp, &gn);
    const float E = hw_sqrt(fmax_nn(U2, 0.0f)) * hw_rcp(R.rf);
    const float f = R.eta_lo * E;
    *vp = gp * f;
    *vn = gn * f;
}

}  // namespace bp
