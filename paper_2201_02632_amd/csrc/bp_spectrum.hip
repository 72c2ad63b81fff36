// K14: flat-sky angular power spectrum of a square map (Sec. 5.3: an FFT of the flat-sky maps,
// logarithmic multipole bins).  F(ell) = d^2 sum_x f(x) e^{-i ell.x} on the modes
// ell = 2 pi (kx, ky) / (N d); the per-mode power |F|^2 / (N d)^2 is averaged over the modes of
// each bin.  A mode's bin is decided on the integer |k|^2 against the edges' |k|^2 in FP64.
//
// The 2-D transform is two passes of one-dimensional FP64 FFTs, one workgroup per line, each line
// held in LDS (N <= 4096 complex doubles = 64 KB): radix-2 decimation in time on bit-reversed input.
//   rows     the real map rows, keeping kx = 0 .. N/2 (the rest is their complex conjugate)
//   T        a tiled transpose, so that each kx column becomes a contiguous line
//   columns  the column transforms; each workgroup bins its column's powers in LDS (FP64 sums,
//            weight 2 for 0 < kx < N/2, whose mirror -kx is not stored) and writes one row of
//            per-column partial sums
//   bins     one workgroup per bin sums the columns' partials in a fixed order.
#include <hip/hip_runtime.h>
#include <math.h>

#include "bp_device.hpp"
#include "bp_internal.hpp"

namespace bp {

constexpr int kSpecMaxN = 4096;
constexpr int kSpecMaxBins = 64;
constexpr int kFftThreads = 256;

struct SpecBins {
    double t[kSpecMaxBins + 1];   // |k|^2 at the bin edges
    int nb;
};

// tw[t] = exp(-2 pi i t / N), t < N/2
__global__ void k_fft_twiddles(int N, double2 *__restrict__ tw) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N / 2) return;
    double s, c;
    sincospi(2.0 * (double)t / (double)N, &s, &c);
    tw[t] = make_double2(c, -s);
}

// in-place transform of buf[0..N) (already in bit-reversed order); ends with a barrier
__device__ inline void fft_lds(double2 *buf, int N, int logN, const double2 *__restrict__ tw) {
    for (int s = 1; s <= logN; ++s) {
        const int half = 1 << (s - 1), step = N >> s;
        for (int t = threadIdx.x; t < N / 2; t += kFftThreads) {
            const int pos = t & (half - 1);
            const int i0 = ((t >> (s - 1)) << s) + pos, i1 = i0 + half;
            const double2 w = tw[pos * step];
            const double2 u = buf[i0], x = buf[i1];
            const double2 v = make_double2(x.x * w.x - x.y * w.y, x.x * w.y + x.y * w.x);
            buf[i0] = make_double2(u.x + v.x, u.y + v.y);
            buf[i1] = make_double2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
}

__device__ inline int bitrev(int i, int logN) { return (int)(__brev((unsigned)i) >> (32 - logN)); }

// rows: A[j][kx] = sum_i f[j][i] e^{-2 pi i kx i / N}, kx = 0 .. N/2
__global__ void __launch_bounds__(kFftThreads) k_fft_rows(int N, int logN, const float *__restrict__ f,
                                                          const double2 *__restrict__ tw, double2 *__restrict__ A) {
    __shared__ double2 buf[kSpecMaxN];
    const int j = blockIdx.x, H = N / 2 + 1;
    for (int i = threadIdx.x; i < N; i += kFftThreads)
        buf[bitrev(i, logN)] = make_double2((double)f[(int64_t)j * N + i], 0.0);
    __syncthreads();
    fft_lds(buf, N, logN, tw);
    for (int k = threadIdx.x; k < H; k += kFftThreads) A[(int64_t)j * H + k] = buf[k];
}

// B[kx][j] = A[j][kx] through 32 x 32 tiles in LDS
__global__ void __launch_bounds__(256) k_transpose_c(int rows, int cols, const double2 *__restrict__ A,
                                                     double2 *__restrict__ B) {
    __shared__ double2 tile[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int rr = r0 + r, cc = c0 + tx;
        if (rr < rows && cc < cols) tile[r][tx] = A[(int64_t)rr * cols + cc];
    }
    __syncthreads();
    for (int c = ty; c < 32; c += 8) {
        const int cc = c0 + c, rr = r0 + tx;
        if (cc < cols && rr < rows) B[(int64_t)cc * rows + rr] = tile[tx][c];
    }
}

// columns: the transform of line kx of B, its powers binned; part[kx][b] = (sum w P, sum w, sum w |k|)
__global__ void __launch_bounds__(kFftThreads) k_fft_cols_power(int N, int logN, const double2 *__restrict__ B,
                                                                const double2 *__restrict__ tw, SpecBins bins,
                                                                double *__restrict__ part) {
    __shared__ double2 buf[kSpecMaxN];
    __shared__ double acc[3 * kSpecMaxBins];
    const int kx = blockIdx.x, nb = bins.nb;
    for (int b = threadIdx.x; b < 3 * nb; b += kFftThreads) acc[b] = 0.0;
    for (int i = threadIdx.x; i < N; i += kFftThreads) buf[bitrev(i, logN)] = B[(int64_t)kx * N + i];
    __syncthreads();
    fft_lds(buf, N, logN, tw);
    const double w = (kx == 0 || 2 * kx == N) ? 1.0 : 2.0;
    for (int k = threadIdx.x; k < N; k += kFftThreads) {
        const int ky = k < N / 2 ? k : k - N;
        const double k2 = (double)(kx * kx + ky * ky);
        if (!(k2 >= bins.t[0] && k2 < bins.t[nb])) continue;
        int lo = 0, hi = nb;                 // the b with t[b] <= k2 < t[b + 1]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (k2 >= bins.t[mid]) lo = mid;
            else hi = mid;
        }
        const double2 F = buf[k];
        unsafeAtomicAdd(&acc[3 * lo], w * (F.x * F.x + F.y * F.y));
        unsafeAtomicAdd(&acc[3 * lo + 1], w);
        unsafeAtomicAdd(&acc[3 * lo + 2], w * sqrt(k2));
    }
    __syncthreads();
    for (int b = threadIdx.x; b < 3 * nb; b += kFftThreads) part[(int64_t)kx * 3 * nb + b] = acc[b];
}

// bins: C_b = d^2 / N^2 * sum P / n_b,  ell_b = 2 pi / (N d) * sum |k| / n_b.  One workgroup per bin;
// lane l sums the columns l, l + 256, ... in order, then a fixed tree over the lanes.
__global__ void __launch_bounds__(256) k_spectrum_bins(int H, int nb, const double *__restrict__ part, double norm,
                                                       double kscale, double *__restrict__ ell,
                                                       double *__restrict__ cl, int64_t *__restrict__ nmodes) {
    __shared__ double r[3][256];
    const int b = blockIdx.x;
    double sp = 0.0, sn = 0.0, sk = 0.0;
    for (int kx = threadIdx.x; kx < H; kx += 256) {
        const double *q = part + (int64_t)kx * 3 * nb + 3 * b;
        sp += q[0];
        sn += q[1];
        sk += q[2];
    }
    r[0][threadIdx.x] = sp;
    r[1][threadIdx.x] = sn;
    r[2][threadIdx.x] = sk;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int c = 0; c < 3; ++c) r[c][threadIdx.x] += r[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sp = r[0][0];
        sn = r[1][0];
        sk = r[2][0];
        nmodes[b] = (int64_t)sn;
        cl[b] = sn > 0.0 ? norm * sp / sn : 0.0;
        ell[b] = sn > 0.0 ? kscale * sk / sn : 0.0;
    }
}

}  // namespace bp

using namespace bp;

extern "C" int bp_flat_power_spectrum(int32_t npix, double pix_rad, const float *map, int32_t nbins,
                                      const double *edges, double *ell, double *cl, int64_t *nmodes, void *ws,
                                      size_t ws_bytes, size_t *ws_needed, void *stream) {
    if (!ws_needed || npix < 2 || npix > kSpecMaxN || (npix & (npix - 1)) || !(pix_rad > 0) || nbins < 1 ||
        nbins > kSpecMaxBins || !edges || !map || !ell || !cl || !nmodes)
        return BP_E_ARG;
    SpecBins bins;
    bins.nb = nbins;
    for (int b = 0; b <= nbins; ++b) {
        if (!(edges[b] >= 0.0) || !isfinite(edges[b]) || (b && !(edges[b] > edges[b - 1]))) return BP_E_ARG;
        const double t = edges[b] * (double)npix * pix_rad / (2.0 * kPi);
        bins.t[b] = t * t;
    }
    const int N = npix, H = N / 2 + 1;
    int logN = 0;
    while ((1 << logN) < N) ++logN;
    Arena S(nullptr, 0);
    S.take<double2>(N / 2 > 0 ? N / 2 : 1); S.take<double2>((size_t)N * H); S.take<double2>((size_t)N * H);
    S.take<double>((size_t)H * 3 * nbins);
    if (!ws || ws_bytes < S.used) { *ws_needed = S.used; return BP_E_WORKSPACE; }
    *ws_needed = S.used;
    Arena A(ws, ws_bytes);
    double2 *tw = A.take<double2>(N / 2 > 0 ? N / 2 : 1);
    double2 *rows = A.take<double2>((size_t)N * H), *cols = A.take<double2>((size_t)N * H);
    double *part = A.take<double>((size_t)H * 3 * nbins);
    hipStream_t s = (hipStream_t)stream;
    prof_begin(BP_PROF_SPECTRUM, s);
    hipLaunchKernelGGL(k_fft_twiddles, dim3((N / 2 + 255) / 256), dim3(256), 0, s, N, tw);
    hipLaunchKernelGGL(k_fft_rows, dim3(N), dim3(kFftThreads), 0, s, N, logN, map, tw, rows);
    hipLaunchKernelGGL(k_transpose_c, dim3((H + 31) / 32, (N + 31) / 32), dim3(256), 0, s, N, H, rows, cols);
    hipLaunchKernelGGL(k_fft_cols_power, dim3(H), dim3(kFftThreads), 0, s, N, logN, cols, tw, bins, part);
    hipLaunchKernelGGL(k_spectrum_bins, dim3(nbins), dim3(256), 0, s, H, nbins, part,
                       pix_rad * pix_rad / ((double)N * (double)N), 2.0 * kPi / ((double)N * pix_rad), ell, cl,
                       nmodes);
    prof_end(BP_PROF_SPECTRUM, s);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}
