// Per-pixel evaluation of a halo's projected footprint from its zone tables
// (shared by the flat-sky and HEALPix deposits).
#pragma once

#include <hip/hip_runtime.h>

#include "bp_device.hpp"

namespace bp {

// Two tables (P and n) sampled at the same position.
__device__ inline void lagr4x2(const float *__restrict__ tp, const float *__restrict__ tn, int n, float s, float *vp,
                               float *vn) {
    float fi = floorf(s);
    int i = (int)fi;
    i = min(max(i, 1), n - 3);
    float f = s - (float)i;
    float fm1 = f - 1.0f, fm2 = f - 2.0f, fp1 = f + 1.0f;
    float w0 = -f * fm1 * fm2 * (1.0f / 6.0f);
    float w1 = fp1 * fm1 * fm2 * 0.5f;
    float w2 = -fp1 * f * fm2 * 0.5f;
    float w3 = fp1 * f * fm1 * (1.0f / 6.0f);
    const float *p = tp + i - 1, *q = tn + i - 1;
    *vp = w0 * p[0] + w1 * p[1] + w2 * p[2] + w3 * p[3];
    *vn = w0 * q[0] + w1 * q[1] + w2 * q[2] + w3 * q[3];
}

__device__ inline void kahan_add(float &s, float &c, float v) {
    float y = v - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Projected profile at squared impact parameter r2 (in the record's length
// unit), in units of the central electron pressure / density times that
// length.  u2 = r_a^2 - r2 and U2 = r_f^2 - r2 are passed in so the caller can
// form them without cancellation next to the footprint edge.
template <class Rec>
__device__ inline void footprint_value(const Rec &R, const float *__restrict__ tab, float r2, float u2, float U2,
                                       float *vp, float *vn) {
    const float *tP = tab, *tN = tab + BP_TAB_ZONE;
    float P = 0.0f, N = 0.0f;
    if (u2 > 0.0f) {
        float u = sqrtf(u2);
        float rr2 = fmaxf(r2, R.r2min);
        float xi = __logf(R.ra + u) - 0.5f * __logf(rr2);
        float eta = log1pf(fmaxf(xi, 0.0f));
        float gp, gn;
        lagr4x2(tP, tN, BP_TAB_NA, (eta - R.eta_lo) * R.eta_ih, &gp, &gn);
        P = gp * u; N = gn * u;
        if (R.flags & 1) {
            float S = sqrtf(u * u + R.D);
            float om = __logf((u + S) / R.sqD);
            float sp, sn;
            lagr4x2(tP + BP_TAB_NA, tN + BP_TAB_NA, BP_TAB_NS, (om - R.om_lo) * R.om_ih, &sp, &sn);
            float e = R.D / (S + u);
            P += sp * e; N += sn * e;
        }
    } else {
        float U = sqrtf(fmaxf(U2, 0.0f));
        float ze = __logf(R.rf + U) - 0.5f * __logf(r2);
        float gp, gn;
        lagr4x2(tP + BP_TAB_NA + BP_TAB_NS, tN + BP_TAB_NA + BP_TAB_NS, BP_TAB_NB, (ze - R.ze_lo) * R.ze_ih, &gp, &gn);
        P = gp * U; N = gn * U;
    }
    *vp = P; *vn = N;
}


// Surrogate tables: 64 nodes per quantity at q_k = (1 - cos(pi k/63))/2, q = r_perp/R_t,
// interpolated in s = acos(1 - 2q)/pi.  R.eta_lo holds R_t and R.eta_ih 1/R_t (record units).
// Y = P_e0 R_t E G(q) with E = sqrt(1 - r_perp^2 / r_f^2) = sqrt(U2) / r_f.
template <class Rec>
__device__ inline void footprint_value_q(const Rec &R, const float *__restrict__ tab, float r2, float U2, float *vp,
                                         float *vn) {
    float q = fminf(sqrtf(r2) * R.eta_ih, 1.0f);
    float sidx = acosf(1.0f - 2.0f * q) * (63.0f / 3.14159265358979f);
    float gp, gn;
    lagr4x2(tab, tab + BP_MLP_NQ, BP_MLP_NQ, sidx, &gp, &gn);
    float E = sqrtf(fmaxf(U2, 0.0f)) / R.rf;
    float f = R.eta_lo * E;
    *vp = gp * f;
    *vn = gn * f;
}

}  // namespace bp
