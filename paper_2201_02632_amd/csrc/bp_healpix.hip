// K9: HEALPix RING ang2pix (Gorski et al. 2005), plus the library's basic
// entry points (version, error strings).
//
// Rings i = 1..4N-1 from the north pole; polar-cap rings hold 4i pixels, belt
// rings 4N.  In the belt (|z| <= 2/3) pixel edges are the lines
// t -+ (3/4) z = const with t = 2 phi / pi, so the two edge-line indices give
// the ring and the position in it; in the caps the edges are the lines
// frac(t) * N sqrt(3(1-|z|)) = const.  The floating-point steps run in FP64 in
// a fixed order with contraction disabled so integer results are reproducible.
#include <hip/hip_runtime.h>
#include <math.h>

#include "bp_device.hpp"
#include "bp_internal.hpp"

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

__global__ void k_ang2pix(int64_t N, int64_t n, const double *__restrict__ th, const double *__restrict__ ph,
                          int64_t *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double t = th[i];
    out[i] = (t >= 0.0 && t <= kPi) ? ang2pix_ring_one(N, t, ph[i]) : -1;
}

}  // namespace bp

using namespace bp;

extern "C" int bp_version(void) { return 100; }

extern "C" const char *bp_strerror(int code) {
    switch (code) {
        case BP_OK: return "ok";
        case BP_E_ARG: return "invalid argument";
        case BP_E_HIP: return "HIP runtime error";
        case BP_E_WORKSPACE: return "workspace too small";
        case BP_E_OVERFLOW: return "size exceeds what one call can index";
        default: return "unknown error";
    }
}

extern "C" int bp_healpix_ang2pix_ring(int64_t nside, int64_t n, const double *theta, const double *phi,
                                       int64_t *ipix, void *stream) {
    if (nside < 1 || nside > (1LL << 29) || n < 0) return BP_E_ARG;
    if (n == 0) return BP_OK;
    if (!theta || !phi || !ipix) return BP_E_ARG;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff) return BP_E_OVERFLOW;
    hipLaunchKernelGGL(k_ang2pix, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, nside, n, theta, phi,
                       ipix);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}
