// K13: particle kSZ onto HEALPix RING pixels by nearest-pixel assignment (App. A of Osato &
// Nagai 2022: the particles of a continuous all-sky light cone are all treated as field particles,
// Eq. field_b, and each amplitude goes whole to the pixel that contains the particle's direction,
// since the SPH footprint of Eq. integrated_kernel needs a regular pixel grid).
//
// The map is cut into tiles of 8192 consecutive RING pixels (a strip of about two rings), small
// enough that one workgroup holds a tile's FP64 sums in LDS.  The particles are bucketed by tile
// with a one-digit counting sort, so no pass uses global atomics:
//   pix      one lane per particle: ang2pix with hardware trigonometry and an error bound; the
//            few directions too close to a pixel edge for that bound are queued in LDS and run
//            through the FP64 reference, so every index equals the pixelisation entry point's.
//            Each block counts its chunk per tile in LDS and writes one row of a [block][tile]
//            count matrix.
//   scan     per tile, prefix sums over groups of blocks, then over tiles: the first slot of every
//            (block, tile) pair in the bucketed entry array.
//   scatter  the same chunks again: amplitude from z and v (an FP32 table of the smooth factor
//            (z / D_A)^2 e^-tau held in LDS), slot from an LDS cursor per tile, entry (pixel within
//            the tile, amplitude) written to its tile's segment.
//   deposit  one workgroup per tile: FP64 sums of the tile's entries in LDS, then one pass over the
//            tile's pixels adding each sum to the FP32 map (one rounding per pixel and call).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include "bp_cosmo.hpp"
#include "bp_device.hpp"
#include "bp_healpix.hpp"
#include "bp_internal.hpp"

namespace bp {

constexpr int kTileBits = 13;
constexpr int kTilePix = 1 << kTileBits;   // pixels per tile (64 KB of FP64 sums)
constexpr int kMaxTiles = 6144;            // 12 * 2048^2 / 8192: nside <= 2048
constexpr int kGroup = 64;                 // blocks per group of the column scan
constexpr int kDepThreads = 1024;
constexpr uint32_t kNoPix = 0xffffffffu;

// RING pixel of one direction without FP64 trigonometry.  The FP64 reference takes a few floors of
// FP64 quantities; here cos(theta) and the cap factor N sin(theta) sqrt(3 / (1 + |z|)) come from the
// hardware sine and cosine, tt = phi / (pi/2) from one FP32 product, and each floor argument
// carries an error bound.  The result is the reference's whenever every argument lies farther than
// its bound from an integer and |z| farther than its bound from 2/3; otherwise the function
// returns false and the caller runs the FP64 reference.  The trigonometric bounds hold over every
// float in [0, pi] with a margin of about 4 (bp_pp_healpix_ngp_selfcheck measures them); the tt
// bound is that of two FP32 roundings.
constexpr float kZErr = 1e-6f;        // |z_hw - cos(theta)|
constexpr double kTmpAbs = 1.5e-6;    // |tmp_hw - tmp| / N, tmp = N sin(theta) sqrt(3 / (1 + |z|))
constexpr double kTmpRel = 2e-7;      // the final product by N
constexpr double kTtRel = 2.5e-7;     // |tt_f32 - tt| / |tt|

__device__ inline double dist_int(double x) { return fabs(x - rint(x)); }

__device__ inline void ngp_trig(int N, float thf, float &zf, float &tmpf) {
#pragma clang fp contract(off)
    zf = __cosf(thf);
    tmpf = (float)N * (__sinf(thf) * __fsqrt_rn(3.0f / (1.0f + fabsf(zf))));
}

// N <= 2048 here, so every ring and pixel index fits in 32 bits and the reference's modulo
// reductions reduce to one conditional add or subtract over the ranges they can take
__device__ inline bool ang2pix_ring_fast(int N, float thf, float phf, int &pix) {
#pragma clang fp contract(off)
    float zf, tmpf;
    ngp_trig(N, thf, zf, tmpf);
    const float zaf = fabsf(zf);
    const float ttf = phf * 0.636619772f;                       // phi / (pi/2)
    const double ett = fabs((double)ttf) * kTtRel + 1e-300;
    const double t4 = (double)ttf * 0.25;
    if (dist_int(t4) <= 0.25 * ett + 1e-15) return false;      // the wrap below must match
    const double tt = (double)ttf - 4.0 * floor(t4);             // exact; |tt - tt_ref| <= ett
    if (fabsf(zaf - 0.6666667f) <= 2.0f * kZErr) return false;
    if (zaf <= 0.6666667f) {
        // belt: a in [N/2, 9N/2), |b| <= N/2, so both floors lie in [0, 5N) and ip in [-N/2, 9N/2 + 1)
        const double a = (double)N * (0.5 + tt);
        const double b = (double)N * ((double)zf * 0.75);
        const double eb = (double)N * (0.75 * (double)kZErr + ett) + 1e-9;
        const double x1 = a - b, x2 = a + b;
        if (dist_int(x1) <= eb || dist_int(x2) <= eb) return false;
        const int asc = (int)floor(x1), dsc = (int)floor(x2);
        const int ir = N + 1 + asc - dsc;
        const int odd = 1 - (ir & 1);
        int ip = (asc + dsc - N + odd + 1) / 2;
        if (ip < 0) ip += 4 * N;
        else if (ip >= 4 * N) ip -= 4 * N;
        pix = 2 * N * (N - 1) + (ir - 1) * 4 * N + ip;
        return true;
    }
    // caps: tt in [0, 4), so floor(tt ir) lies in [0, 4 ir]
    if (dist_int(tt) <= ett + 1e-15) return false;
    const double tf = tt - floor(tt);
    const double ec = (double)N * kTmpAbs + (double)tmpf * (kTmpRel + 1.01 * ett) + 1e-9;
    const double x1 = tf * (double)tmpf, x2 = (1.0 - tf) * (double)tmpf;
    if (dist_int(x1) <= ec || dist_int(x2) <= ec) return false;
    const int ir = (int)floor(x1) + (int)floor(x2) + 1;
    const double xi = tt * (double)ir;
    if (dist_int(xi) <= (double)ir * ett + 1e-9) return false;
    int ip = (int)floor(xi);
    if (ip >= 4 * ir) ip -= 4 * ir;
    pix = zf > 0.0f ? 2 * ir * (ir - 1) + ip : 12 * N * N - 2 * ir * (ir + 1) + ip;
    return true;
}

constexpr int kU = 4;        // particles in flight per lane
constexpr int kQueue = 2048; // per block: directions left for the FP64 reference

// the queued directions of a block through the FP64 reference (all lanes of the block call this)
__device__ inline void ngp_flush(int64_t N, int64_t i0, const float *__restrict__ th, const float *__restrict__ ph,
                                 const uint32_t *queue, int nq, uint32_t *hist, uint32_t *__restrict__ pix) {
    for (int k = threadIdx.x; k < nq; k += 256) {
        const int64_t i = i0 + queue[k];
        const uint32_t p = (uint32_t)ang2pix_ring_one(N, (double)th[i], (double)ph[i]);
        atomicAdd(&hist[p >> kTileBits], 1u);
        pix[i] = p;
    }
}

__global__ void __launch_bounds__(256) k_ngp_pix(int64_t N, int64_t n, int64_t chunk, const float *__restrict__ th,
                                                 const float *__restrict__ ph, int ntiles, uint32_t *__restrict__ pix,
                                                 uint32_t *__restrict__ counts, uint32_t *__restrict__ bad) {
    extern __shared__ uint32_t hist[];
    __shared__ uint32_t queue[kQueue];
    __shared__ int qn;
    for (int t = threadIdx.x; t < ntiles; t += 256) hist[t] = 0u;
    if (threadIdx.x == 0) qn = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = min(n, i0 + chunk);
    int nb = 0;
    for (int64_t round = i0; round < i1; round += 256 * kU) {     // the same trip count on every lane
        const int64_t base = round + threadIdx.x;
        float t[kU], f[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t i = base + u * 256;
            t[u] = i < i1 ? th[i] : 0.0f;
            f[u] = i < i1 ? ph[i] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t i = base + u * 256;
            if (i >= i1) break;
            uint32_t p = kNoPix;
            if ((double)t[u] >= 0.0 && (double)t[u] <= kPi && isfinite(f[u])) {
                int pp;
                if (!ang2pix_ring_fast((int)N, t[u], f[u], pp)) {
                    queue[atomicAdd(&qn, 1)] = (uint32_t)(i - i0);   // at most 256 kU per round: fits
                    continue;
                }
                p = (uint32_t)pp;
                atomicAdd(&hist[p >> kTileBits], 1u);
            } else {
                nb = 1;
            }
            pix[i] = p;
        }
        __syncthreads();
        const int nq = qn;
        __syncthreads();            // every lane has read qn before any lane adds to it again
        if (nq > kQueue - 256 * kU || round + 256 * kU >= i1) {
            ngp_flush(N, i0, th, ph, queue, nq, hist, pix);
            __syncthreads();
            if (threadIdx.x == 0) qn = 0;
            __syncthreads();
        }
    }
    if (nb) atomicOr(bad, 1u);
    __syncthreads();
    uint32_t *row = counts + (int64_t)blockIdx.x * ntiles;
    for (int t = threadIdx.x; t < ntiles; t += 256) row[t] = hist[t];
}

// gs[g][t] = sum of counts[b][t] over the blocks b of group g
__global__ void __launch_bounds__(256) k_ngp_group_sums(int nblk, int ntiles, const uint32_t *__restrict__ counts,
                                                        uint32_t *__restrict__ gs) {
    const int t = blockIdx.x * 256 + threadIdx.x, g = blockIdx.y;
    if (t >= ntiles) return;
    const int b1 = min(nblk, (g + 1) * kGroup);
    uint32_t s = 0;
    for (int b = g * kGroup; b < b1; ++b) s += counts[(int64_t)b * ntiles + t];
    gs[(int64_t)g * ntiles + t] = s;
}

// per tile: exclusive prefix over groups (in place) and the tile total
__global__ void __launch_bounds__(256) k_ngp_group_scan(int ngroups, int ntiles, uint32_t *__restrict__ gs,
                                                        uint32_t *__restrict__ tot) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= ntiles) return;
    uint32_t s = 0;
    for (int g = 0; g < ngroups; ++g) {
        const uint32_t c = gs[(int64_t)g * ntiles + t];
        gs[(int64_t)g * ntiles + t] = s;
        s += c;
    }
    tot[t] = s;
}

// counts[b][t] becomes the first slot of block b in tile t
__global__ void __launch_bounds__(256) k_ngp_offsets(int nblk, int ntiles, uint32_t *__restrict__ counts,
                                                     const uint32_t *__restrict__ gs, const uint32_t *__restrict__ beg) {
    const int t = blockIdx.x * 256 + threadIdx.x, g = blockIdx.y;
    if (t >= ntiles) return;
    const int b1 = min(nblk, (g + 1) * kGroup);
    uint32_t s = beg[t] + gs[(int64_t)g * ntiles + t];
    for (int b = g * kGroup; b < b1; ++b) {
        const uint32_t c = counts[(int64_t)b * ntiles + t];
        counts[(int64_t)b * ntiles + t] = s;
        s += c;
    }
}

// G(z) = (z / D_A(z))^2 e^-tau(z) on a uniform z grid (FP32): smooth down to z = 0, where it is
// (H0/c)^2, so b_i = amp_k v_i G(z_i) / z_i^2 needs only a short table and FP32 arithmetic
constexpr int kNG = 4096;

__global__ void k_ngp_gtable(const double *__restrict__ chi_t, const double *__restrict__ tau_t,
                             float *__restrict__ G) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kNG) return;
    const double z = kZmax * k / (kNG - 1);
    if (k == 0) {
        G[0] = (float)((100.0 / kCkms) * (100.0 / kCkms));
        return;
    }
    const double r = z * (1.0 + z) / table_interp(chi_t, z);
    G[k] = (float)(r * r * exp(-table_interp(tau_t, z)));
}

// Exclusive prefix sum of c[0..m) in place over a block of kSortThreads lanes (m <= 12 kSortThreads);
// returns the total.  Each lane sums a contiguous run of c, the lanes scan their run sums with
// wavefront shuffles and the wavefront totals through LDS.
constexpr int kSortThreads = 512;
constexpr int kSortPer = 8;   // 4096-particle sub-chunks: two blocks per CU (timed against 1024 .. 8192)

__device__ inline uint32_t block_exclusive_scan(uint32_t *c, int m, uint32_t *wtot) {
    const int per = (m + kSortThreads - 1) / kSortThreads;
    const int b0 = threadIdx.x * per, b1 = min(m, b0 + per);
    uint32_t run = 0;
    for (int k = b0; k < b1; ++k) run += c[k];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = run;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) wtot[wave] = inc;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int w = 0; w < kSortThreads / 64; ++w) {
        before += w < wave ? wtot[w] : 0u;
        total += wtot[w];
    }
    uint32_t x = before + inc - run;
    for (int k = b0; k < b1; ++k) {
        const uint32_t v = c[k];
        c[k] = x;
        x += v;
    }
    return total;
}

// amp_k = sigma_T (1 km/s / c) f_gas M_p / (mu_e m_p) / ((Mpc/h)^2 Omega_pix).
// The block walks its chunk in sub-chunks of PER * kSortThreads particles; each sub-chunk is
// counting-sorted by tile in LDS before it is written, so consecutive lanes store consecutive slots
// of a tile's segment instead of 64 unrelated cache lines per wavefront store.
template <int PER>
__global__ void __launch_bounds__(kSortThreads) k_ngp_scatter(int64_t n, int64_t chunk,
                                                              const uint32_t *__restrict__ pix,
                                                              const float *__restrict__ zz,
                                                              const float *__restrict__ vl,
                                                              const float *__restrict__ Gt, float amp_k, int ntiles,
                                                              const uint32_t *__restrict__ offsets,
                                                              uint2 *__restrict__ ent, uint32_t *__restrict__ bad) {
    constexpr int S = PER * kSortThreads;
    extern __shared__ uint32_t lds[];
    float *G = (float *)lds;                              // kNG
    uint32_t *cur = lds + kNG;                            // ntiles: next slot of this block in each tile
    uint32_t *cnt = cur + ntiles;                         // ntiles: counts, then offsets, of a sub-chunk
    uint2 *sent = (uint2 *)(cnt + ntiles + (ntiles & 1)); // S entries in tile order
    uint32_t *sslot = (uint32_t *)(sent + S);             // S global slots
    __shared__ uint32_t wtot[kSortThreads / 64];
    const uint32_t *row = offsets + (int64_t)blockIdx.x * ntiles;
    for (int t = threadIdx.x; t < ntiles; t += kSortThreads) {
        cur[t] = row[t];
        cnt[t] = 0u;
    }
    for (int k = threadIdx.x; k < kNG; k += kSortThreads) G[k] = Gt[k];
    __syncthreads();
    const float gs = (float)((kNG - 1) / kZmax);
    const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = min(n, i0 + chunk);
    int nb = 0;
    for (int64_t sub = i0; sub < i1; sub += S) {          // the same trip count on every lane
        uint32_t tl[PER], rk[PER];
        uint2 e[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int64_t i = sub + u * kSortThreads + threadIdx.x;
            uint32_t p = kNoPix;
            float z = 0.0f, v = 0.0f;
            if (i < i1) {
                p = pix[i];
                z = zz[i];
                v = vl[i];
            }
            tl[u] = kNoPix;
            if (p == kNoPix) continue;
            float a = 0.0f;
            if (z >= 0.0f && (double)z < kZmax - 0.01) {
                const float s = z * gs;
                const int j = min(max((int)s, 1), kNG - 3);
                const float x = s - (float)j;
                const float w0 = -x * (x - 1.0f) * (x - 2.0f) * (1.0f / 6.0f);
                const float w1 = (x + 1.0f) * (x - 1.0f) * (x - 2.0f) * 0.5f;
                const float w2 = -(x + 1.0f) * x * (x - 2.0f) * 0.5f;
                const float w3 = (x + 1.0f) * x * (x - 1.0f) * (1.0f / 6.0f);
                const float g = w0 * G[j - 1] + w1 * G[j] + w2 * G[j + 1] + w3 * G[j + 2];
                a = amp_k * v * g / (z * z);
            } else {
                nb = 1;
            }
            tl[u] = p >> kTileBits;
            e[u] = make_uint2(p & (kTilePix - 1), __float_as_uint(a));
        }
#pragma unroll
        for (int u = 0; u < PER; ++u)
            if (tl[u] != kNoPix) rk[u] = atomicAdd(&cnt[tl[u]], 1u);
        __syncthreads();
        const uint32_t m = block_exclusive_scan(cnt, ntiles, wtot);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            if (tl[u] == kNoPix) continue;
            const uint32_t k = cnt[tl[u]] + rk[u];
            sent[k] = e[u];
            sslot[k] = cur[tl[u]] + rk[u];
        }
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < m; k += kSortThreads) ent[sslot[k]] = sent[k];
        // advance the cursors by this sub-chunk's counts and clear the counters
        uint32_t adv[(6144 + kSortThreads - 1) / kSortThreads];
        int na = 0;
        for (int t = threadIdx.x; t < ntiles; t += kSortThreads)
            adv[na++] = (t + 1 < ntiles ? cnt[t + 1] : m) - cnt[t];
        __syncthreads();
        na = 0;
        for (int t = threadIdx.x; t < ntiles; t += kSortThreads) {
            cur[t] += adv[na++];
            cnt[t] = 0u;
        }
        __syncthreads();
    }
    if (nb) atomicOr(bad, 1u);
}

size_t scatter_lds_bytes(int per, int ntiles) {
    return sizeof(float) * kNG + sizeof(uint32_t) * (2 * (size_t)ntiles + (ntiles & 1)) +
           (size_t)per * kSortThreads * (sizeof(uint2) + sizeof(uint32_t));
}

__global__ void __launch_bounds__(kDepThreads) k_ngp_deposit(int64_t npix, const uint32_t *__restrict__ beg,
                                                             const uint2 *__restrict__ ent, float *__restrict__ map) {
    __shared__ double acc[kTilePix];
    const int t = blockIdx.x;
    const uint32_t e0 = beg[t], e1 = beg[t + 1];
    if (e0 == e1) return;
    for (int k = threadIdx.x; k < kTilePix; k += kDepThreads) acc[k] = 0.0;
    __syncthreads();
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += kDepThreads * kU) {
        uint2 q[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) q[u] = e + u * kDepThreads < e1 ? ent[e + u * kDepThreads] : make_uint2(0u, 0u);
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if (e + u * kDepThreads < e1) unsafeAtomicAdd(&acc[q[u].x], (double)__uint_as_float(q[u].y));
    }
    __syncthreads();
    const int64_t p0 = (int64_t)t << kTileBits;
    const int m = (int)min((int64_t)kTilePix, npix - p0);
    for (int k = threadIdx.x; k < m; k += kDepThreads) {
        const double a = acc[k];
        if (a != 0.0) map[p0 + k] = (float)((double)map[p0 + k] + a);
    }
}

// Over every float theta in [0, pi): max |z_hw - cos| and max |tmp_hw - tmp| / N where |cos| > 0.66,
// against FP64 cos, sin and sqrt (as ordered integers of the non-negative float errors)
__global__ void k_ngp_trig_check(int N, uint32_t last, uint32_t *__restrict__ out) {
    uint32_t mz = 0u, mt = 0u;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k <= last; k += gridDim.x * blockDim.x) {
        const float t = __uint_as_float(k);
        float zf, tmpf;
        ngp_trig(N, t, zf, tmpf);
        const double zd = cos((double)t);
        mz = max(mz, __float_as_uint((float)fabs((double)zf - zd)));
        if (fabs(zd) > 0.66) {
            const double td = (double)N * (sin((double)t) * sqrt(3.0 / (1.0 + fabs(zd))));
            mt = max(mt, __float_as_uint((float)(fabs((double)tmpf - td) / (double)N)));
        }
    }
    atomicMax(&out[0], mz);
    atomicMax(&out[1], mt);
}

}  // namespace bp

using namespace bp;

extern "C" int bp_pp_healpix_ngp_selfcheck(int64_t nside, double *bounds, void *ws, size_t ws_bytes,
                                           size_t *ws_needed, void *stream) {
    if (nside < 1 || nside > 2048 || !bounds || !ws_needed) return BP_E_ARG;
    const size_t need = 256;   // two uint32 maxima, rounded as the workspace arena rounds
    *ws_needed = need;
    if (!ws || ws_bytes < need) return BP_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    uint32_t *d = (uint32_t *)ws;
    int e = fill_u32(d, 0u, 2, s);
    const float pi_below = 3.14159250f;   // the largest float below pi
    uint32_t last;
    memcpy(&last, &pi_below, sizeof(last));
    if (!e) {
        hipLaunchKernelGGL(k_ngp_trig_check, dim3(4096), dim3(256), 0, s, (int)nside, last, d);
        if (hipGetLastError() != hipSuccess) e = BP_E_HIP;
    }
    uint32_t h[2] = {0u, 0u};
    if (!e && hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) e = BP_E_HIP;
    if (!e && hipStreamSynchronize(s) != hipSuccess) e = BP_E_HIP;
    if (e) return e;
    float f[2];
    memcpy(f, h, sizeof(f));
    bounds[0] = f[0];
    bounds[1] = f[1];
    bounds[2] = kZErr;
    bounds[3] = kTmpAbs;
    return BP_OK;
}

extern "C" int bp_pp_paste_healpix_ngp(const bp_params *p, int64_t nside, int64_t n, const float *theta,
                                       const float *phi, const float *z, const float *v_los, double M_p,
                                       float *b_map, void *ws, size_t ws_bytes, size_t *ws_needed, void *stream) {
    if (check_params(p) || nside < 1 || nside > 2048 || n < 0 || !ws_needed || !(M_p > 0) || !b_map) return BP_E_ARG;
    if (n == 0) { *ws_needed = 0; return BP_OK; }
    if (!theta || !phi || !z || !v_los) return BP_E_ARG;
    if (n >= 0x7fffffffLL) return BP_E_OVERFLOW;
    hipStream_t s = (hipStream_t)stream;
    const int64_t npix = 12 * nside * nside;
    const int ntiles = (int)((npix + kTilePix - 1) >> kTileBits);
    if (ntiles > kMaxTiles) return BP_E_ARG;
    // chunk per block: about 4096 blocks for large inputs, at least 4096 particles each
    int64_t chunk = ((n + 4095) / 4096 + 255) / 256 * 256;
    chunk = chunk < 4096 ? 4096 : (chunk > 65536 ? 65536 : chunk);
    const int nblk = (int)((n + chunk - 1) / chunk);
    const int ngroups = (nblk + kGroup - 1) / kGroup;

    Arena S(nullptr, 0);
    S.take<double>(kNZ); S.take<double>(kNZ);
    S.take<uint32_t>(n); S.take<uint32_t>((size_t)nblk * ntiles); S.take<uint32_t>((size_t)ngroups * ntiles);
    S.take<uint32_t>(ntiles + 1); S.take<uint32_t>(ntiles + 1); S.take<uint32_t>(1); S.take<float>(kNG);
    S.take<uint2>(n);
    const size_t need = S.used + scan_ws_bytes(ntiles + 1);
    if (!ws || ws_bytes < need) { *ws_needed = need; return BP_E_WORKSPACE; }
    *ws_needed = need;
    Arena A(ws, ws_bytes);
    double *chi_t = A.take<double>(kNZ), *tau_t = A.take<double>(kNZ);
    uint32_t *pix = A.take<uint32_t>(n);
    uint32_t *counts = A.take<uint32_t>((size_t)nblk * ntiles);
    uint32_t *gs = A.take<uint32_t>((size_t)ngroups * ntiles);
    uint32_t *tot = A.take<uint32_t>(ntiles + 1), *beg = A.take<uint32_t>(ntiles + 1);
    uint32_t *bad = A.take<uint32_t>(1);
    float *Gt = A.take<float>(kNG);
    uint2 *ent = A.take<uint2>(n);
    void *scan_ws = (char *)ws + A.used;

    const double u_len = kMpc / p->h, Mp_g = M_p * kMsun / p->h, mu_e = 2.0 / (1.0 + p->X_H);
    const double omega_pix = 4.0 * kPi / (double)npix;
    const float amp_k =
        (float)(kSigmaT * (1e5 / kC) * (p->field_gas_frac * Mp_g / (mu_e * kMp)) / (u_len * u_len * omega_pix));
    const size_t lds = (size_t)ntiles * sizeof(uint32_t);
    const unsigned tiles_x = (unsigned)((ntiles + 255) / 256);

    prof_begin(BP_PROF_NGP_PLAN, s);
    int e = cosmo_tables(*p, chi_t, tau_t, s);
    if (!e && (fill_u32(bad, 0u, 1, s) || fill_u32(tot + ntiles, 0u, 1, s))) e = BP_E_HIP;
    if (e) return e;
    hipLaunchKernelGGL(k_ngp_gtable, dim3(kNG / 256), dim3(256), 0, s, chi_t, tau_t, Gt);
    hipLaunchKernelGGL(k_ngp_pix, dim3((unsigned)nblk), dim3(256), lds, s, nside, n, chunk, theta, phi, ntiles, pix,
                       counts, bad);
    hipLaunchKernelGGL(k_ngp_group_sums, dim3(tiles_x, (unsigned)ngroups), dim3(256), 0, s, nblk, ntiles, counts, gs);
    hipLaunchKernelGGL(k_ngp_group_scan, dim3(tiles_x), dim3(256), 0, s, ngroups, ntiles, gs, tot);
    if (hipGetLastError() != hipSuccess) return BP_E_HIP;
    e = scan_exclusive_u32(tot, beg, ntiles + 1, scan_ws, s);
    if (e) return e;
    hipLaunchKernelGGL(k_ngp_offsets, dim3(tiles_x, (unsigned)ngroups), dim3(256), 0, s, nblk, ntiles, counts, gs,
                       beg);
    const size_t slds = scatter_lds_bytes(kSortPer, ntiles);   // above 64 KB: raise the kernel's limit
    if (hipFuncSetAttribute((const void *)k_ngp_scatter<kSortPer>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)slds) != hipSuccess)
        return BP_E_HIP;
    hipLaunchKernelGGL(k_ngp_scatter<kSortPer>, dim3((unsigned)nblk), dim3(kSortThreads), slds, s, n, chunk, pix, z,
                       v_los, Gt, amp_k, ntiles, counts, ent, bad);
    prof_end(BP_PROF_NGP_PLAN, s);
    if (hipGetLastError() != hipSuccess) return BP_E_HIP;
    uint32_t hbad = 0;
    if (hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, s) != hipSuccess) return BP_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return BP_E_HIP;
    if (hbad) return BP_E_ARG;
    prof_begin(BP_PROF_NGP_DEPOSIT, s);
    hipLaunchKernelGGL(k_ngp_deposit, dim3((unsigned)ntiles), dim3(kDepThreads), 0, s, npix, beg, ent, b_map);
    prof_end(BP_PROF_NGP_DEPOSIT, s);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}
