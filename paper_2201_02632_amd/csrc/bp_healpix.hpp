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

__host__ __device__ inline int64_t ang2pix_ring_one(int64_t N, double theta, double phi) {
#pragma clang fp contract(off)
    const double halfpi = 1.5707963267948966;
    double z = cos(theta), za = fabs(z);
    double tt = phi / halfpi;
    tt = tt - 4.0 * floor(tt / 4.0);
    if (tt >= 4.0) tt = 0.0;
    if (za <= 2.0 / 3.0) {
        double a = (double)N * (0.5 + tt);
        double b = (double)N * (z * 0.75);
        int64_t asc = (int64_t)floor(a - b);
        int64_t dsc = (int64_t)floor(a + b);
        int64_t ir = N + 1 + asc - dsc;                 // ring counted from z = 2/3, 1..2N+1
        int64_t odd = 1 - (ir & 1);
        int64_t ip = (asc + dsc - N + odd + 1) / 2;     // numerator is >= 0 here
        ip = ((ip % (4 * N)) + 4 * N) % (4 * N);
        return 2 * N * (N - 1) + (ir - 1) * 4 * N + ip;
    }
    double tf = tt - floor(tt);
    double s = sin(theta);
    double tmp = (double)N * (s * sqrt(3.0 / (1.0 + za)));  // N sqrt(3(1-|z|)) without cancellation
    int64_t jp = (int64_t)floor(tf * tmp);
    int64_t jm = (int64_t)floor((1.0 - tf) * tmp);
    int64_t ir = jp + jm + 1;                               // ring counted from the nearer pole
    int64_t ip = (int64_t)floor(tt * (double)ir);
    ip = ((ip % (4 * ir)) + 4 * ir) % (4 * ir);
    if (z > 0) return 2 * ir * (ir - 1) + ip;
    return 12 * N * N - 2 * ir * (ir + 1) + ip;
}

}  // namespace bp
