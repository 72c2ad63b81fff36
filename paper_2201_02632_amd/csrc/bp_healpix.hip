// K9: HEALPix RING ang2pix (Gorski et al. 2005; the per-direction arithmetic is in
// bp_healpix.hpp), plus the library's basic entry points (version, error strings).
#include <hip/hip_runtime.h>
#include <math.h>

#include "bp_device.hpp"
#include "bp_healpix.hpp"
#include "bp_internal.hpp"

namespace bp {

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
