// HEALPix RING ang2pix (Gorski et al. 2005), shared by the pixelisation entry point and the
// all-sky particle paste.
//
// Rings i = 1..4N-1 from the north pole; polar-cap rings hold 4i pixels, belt
// rings 4N.  In the belt (|z| <= 2/3) pixel edges are the lines
// t -+ (3/4) z = const with t = 2 phi / pi, so the two edge-line indices give
// the ring and the position in it; in the caps the edges are the lines
// frac(t) * N sqrt(3(1-|z|)) = const.  The floating-point steps run in FP64 in
// a fixed order with contraction disabled so integer results are reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace bp {

// ---- cos and sin of a colatitude rounded correctly to FP64 --------------------------------------
// Pixel indices are decided by floors of products of cos(theta) and sin(theta); next to a pixel edge
// the last bit of either can move the index, and the device's cos / sin are not always the correctly
// rounded values.  For those few directions both are recomputed in double-double arithmetic (sums and
// products with their exact rounding errors, Dekker / Knuth), the argument reduced by a double-double
// pi / 2 and the Taylor series summed to x^29 on |x| <= pi / 4 (remainder below 1e-30 relative), and
// rounded once.
struct DD { double hi, lo; };
__host__ __device__ inline DD dd_quick(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    return {s, b - (s - a)};
}
__host__ __device__ inline DD dd_sum(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b, bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
__host__ __device__ inline DD dd_add(DD a, DD b) {
#pragma clang fp contract(off)
    DD s = dd_sum(a.hi, b.hi), t = dd_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = dd_quick(s.hi, s.lo);
    s.lo += t.lo;
    return dd_quick(s.hi, s.lo);
}
__host__ __device__ inline DD dd_mul(DD a, DD b) {
#pragma clang fp contract(off)
    const double p = a.hi * b.hi;
    double e = fma(a.hi, b.hi, -p);
    e += a.hi * b.lo + a.lo * b.hi;
    return dd_quick(p, e);
}
__host__ __device__ inline DD dd_div_small(DD a, double b) {   // a / b for a small integer b
#pragma clang fp contract(off)
    const double q = a.hi / b;
    const double p = q * b, pe = fma(q, b, -p);
    const double r = ((a.hi - p) - pe + a.lo) / b;
    return dd_quick(q, r);
}
__host__ __device__ inline void cos_sin_cr(double theta, double *c, double *s) {
    const DD halfpi = {1.5707963267948966, 6.123233995736766e-17};
    const int k = (int)floor(theta / halfpi.hi + 0.5);              // 0, 1 or 2 for theta in [0, pi]
    // theta - k pi/2: theta - k halfpi.hi is exact here (k halfpi.hi lies within a factor 2 of theta)
    const DD x = dd_add({theta - k * halfpi.hi, 0.0}, {-k * halfpi.lo, 0.0});
    const DD x2 = dd_mul(x, x);
    DD sn = x, cs = {1.0, 0.0}, ts = x, tc = {1.0, 0.0};
    for (int j = 1; j <= 14; ++j) {
        tc = dd_div_small(dd_mul(tc, {-x2.hi, -x2.lo}), (double)((2 * j - 1) * (2 * j)));
        ts = dd_div_small(dd_mul(ts, {-x2.hi, -x2.lo}), (double)((2 * j) * (2 * j + 1)));
        cs = dd_add(cs, tc);
        sn = dd_add(sn, ts);
    }
    const double sx = sn.hi + sn.lo, cx = cs.hi + cs.lo;            // normalised: these are the rounded values
    if (k == 0) { *c = cx; *s = sx; }
    else if (k == 1) { *c = -sx; *s = cx; }
    else { *c = -cx; *s = -sx; }
}

// a floor argument within 1e-8 of an integer: far above the error of the device's cos / sin there
__host__ __device__ inline bool near_int(double v) {
    const double f = v - floor(v);
    return f < 1e-8 || f > 1.0 - 1e-8;
}

// RING index from z = cos(theta), s = sin(theta) and t = phi / (pi/2) in [0, 4); *edge is set when the
// result could depend on the last bit of z or s
__host__ __device__ inline int64_t ring_pixel(int64_t N, double z, double s, double tt, bool *edge) {
#pragma clang fp contract(off)
    const double za = fabs(z);
    if (za <= 2.0 / 3.0) {
        double a = (double)N * (0.5 + tt);
        double b = (double)N * (z * 0.75);
        *edge = near_int(a - b) || near_int(a + b) || fabs(za - 2.0 / 3.0) < 1e-14;
        int64_t asc = (int64_t)floor(a - b);
        int64_t dsc = (int64_t)floor(a + b);
        int64_t ir = N + 1 + asc - dsc;                 // ring counted from z = 2/3, 1..2N+1
        int64_t odd = 1 - (ir & 1);
        int64_t ip = (asc + dsc - N + odd + 1) / 2;     // numerator is >= 0 here
        ip = ((ip % (4 * N)) + 4 * N) % (4 * N);
        return 2 * N * (N - 1) + (ir - 1) * 4 * N + ip;
    }
    double tf = tt - floor(tt);
    double tmp = (double)N * (s * sqrt(3.0 / (1.0 + za)));  // N sqrt(3(1-|z|)) without cancellation
    *edge = near_int(tf * tmp) || near_int((1.0 - tf) * tmp) || fabs(za - 2.0 / 3.0) < 1e-14;
    int64_t jp = (int64_t)floor(tf * tmp);
    int64_t jm = (int64_t)floor((1.0 - tf) * tmp);
    int64_t ir = jp + jm + 1;                               // ring counted from the nearer pole
    int64_t ip = (int64_t)floor(tt * (double)ir);
    ip = ((ip % (4 * ir)) + 4 * ir) % (4 * ir);
    if (z > 0) return 2 * ir * (ir - 1) + ip;
    return 12 * N * N - 2 * ir * (ir + 1) + ip;
}

// The pixel of the direction (theta, phi) whose cos(theta) and sin(theta) are rounded correctly to
// FP64 (theta in [0, pi], phi any finite value).
__host__ __device__ inline int64_t ang2pix_ring_one(int64_t N, double theta, double phi) {
#pragma clang fp contract(off)
    const double halfpi = 1.5707963267948966;
    double tt = phi / halfpi;
    tt = tt - 4.0 * floor(tt / 4.0);
    if (tt >= 4.0) tt = 0.0;
    bool edge = false;
    const int64_t p = ring_pixel(N, cos(theta), sin(theta), tt, &edge);
    if (!edge) return p;
    double z, s;
    cos_sin_cr(theta, &z, &s);
    return ring_pixel(N, z, s, tt, &edge);
}

}  // namespace bp
