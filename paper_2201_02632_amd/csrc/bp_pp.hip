// Particle-based pasting (Sec. 3.4 of Osato & Nagai 2022).
//
// K5  cell sort: comoving Cartesian positions (chi theta_x, chi theta_y, chi)
//     are binned on a dense grid of coarse cells; inside a coarse cell the
//     particles are ordered by a 30-bit Morton code of their position, so the
//     key (coarse cell << 30 | Morton) makes every cell of every finer level a
//     contiguous, binary-searchable run of the sorted arrays.
// K6  kNN: one lane per particle (in sorted order, so a wavefront works on
//     neighbouring particles).  At level l it scans the 3x3x3 block of level-l
//     cells around the particle, keeping the k smallest squared distances in
//     registers; the k-th distance is exact once it does not exceed the cell
//     size (everything outside the block is at least one cell away).  The
//     start level comes from the coarse-cell occupancy, so dense halo cores
//     and empty voids both scan a few hundred candidates.
// K7  per-particle signal amplitudes and angular smoothing lengths.
// K8  separable SPH deposit: the particle's weight on pixel (i, j) is the
//     product of one-dimensional integrated-kernel differences.  Particles are
//     split by footprint width: narrow ones onto 16x16 tiles (one wavefront per
//     tile), wide ones onto 64x64 tiles (one workgroup per tile, the per-axis
//     weights staged in LDS).  Each pixel is owned by one lane and summed with
//     Kahan compensation in a fixed order, as in the halo deposit.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>

#include "bp_cosmo.hpp"
#include "bp_device.hpp"
#include "bp_internal.hpp"

namespace bp {

// ------------------------------------------------------ cosmology tables --
// chi(z)/(c/H0) and the optical-depth integral on a uniform z grid (24-point GL per cell from the previous node)
__global__ void k_cosmo_table(bp_params P, GaussRules G, double *__restrict__ chi_t, double *__restrict__ tau_t) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNZ) return;
    double z = kZmax * i / (kNZ - 1);
    double a1 = 0.0, a2 = 0.0;
    for (int j = 0; j < 24; ++j) {
        double zz = 0.5 * z * (G.x24[j] + 1.0), zp = 1.0 + zz;
        double E = sqrt(P.Omega_m * zp * zp * zp + 1.0 - P.Omega_m);
        a1 += G.w24[j] / E;
        a2 += G.w24[j] * zp * zp / E;
    }
    double cH = kCkms / 100.0;
    double H0 = 100.0 * P.h * 1e5 / kMpc;
    double rho_cr0 = 3.0 * H0 * H0 / (8.0 * kPi * kG);
    double ne_bar = P.Omega_b * rho_cr0 / (2.0 / (1.0 + P.X_H) * kMp);
    chi_t[i] = cH * 0.5 * z * a1;
    tau_t[i] = kSigmaT * ne_bar * (kC / H0) * 0.5 * z * a2;
}

int cosmo_tables(const bp_params &P, double *chi_t, double *tau_t, hipStream_t s) {
    hipLaunchKernelGGL(k_cosmo_table, dim3((kNZ + 255) / 256), dim3(256), 0, s, P, gauss_rules(), chi_t, tau_t);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

// ------------------------------------------------------------- K5 sort --
struct Grid {
    double x0, y0, z0;   // origin of the coarse grid (comoving Mpc/h)
    double cell;         // coarse cell size
    int32_t nx, ny, nz;
    int64_t ncells;
};

__device__ inline uint32_t spread10(uint32_t v) {  // 10 bits -> every third bit
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__device__ inline uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    return spread10(x) | (spread10(y) << 1) | (spread10(z) << 2);
}

// positions and bounding box (min/max reduced with atomics on ordered integer images of doubles)
__device__ inline unsigned long long dbl_order(double v) {
    unsigned long long u = __double_as_longlong(v);
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}
__device__ inline double dbl_unorder(unsigned long long u) {
    u = (u & 0x8000000000000000ull) ? (u & 0x7fffffffffffffffull) : ~u;
    return __longlong_as_double(u);
}

__global__ void __launch_bounds__(256) k_pp_positions(int64_t n, const float *__restrict__ tx, const float *__restrict__ ty,
                                                      const float *__restrict__ zz, const double *__restrict__ chi_t,
                                                      double *__restrict__ pos, unsigned long long *__restrict__ bbox,
                                                      int *__restrict__ bad) {
    // grid-stride over particles with a capped grid, so the bounding box costs one atomic per block and axis
    unsigned long long lo[3] = {~0ull, ~0ull, ~0ull}, hi[3] = {0ull, 0ull, 0ull};
    int nbad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double z = zz[i];
        double X = 0, Y = 0, Z = 0;
        const bool ok = z >= 0.0 && z < kZmax - 0.01 && isfinite((double)tx[i]) && isfinite((double)ty[i]);
        if (ok) {
            double chi = table_interp(chi_t, z);
            X = chi * (double)tx[i]; Y = chi * (double)ty[i]; Z = chi;
            const unsigned long long o[3] = {dbl_order(X), dbl_order(Y), dbl_order(Z)};
            for (int a = 0; a < 3; ++a) {
                lo[a] = o[a] < lo[a] ? o[a] : lo[a];
                hi[a] = o[a] > hi[a] ? o[a] : hi[a];
            }
        } else {
            nbad = 1;
        }
        pos[i] = X; pos[n + i] = Y; pos[2 * n + i] = Z;
    }
    if (nbad) atomicOr(bad, 1);
    __shared__ unsigned long long mn[3][4], mx[3][4];
    for (int a = 0; a < 3; ++a) {
        unsigned long long l = lo[a], h = hi[a];
        for (int o = 32; o > 0; o >>= 1) {
            unsigned long long l2 = __shfl_down(l, o, 64), h2 = __shfl_down(h, o, 64);
            l = l2 < l ? l2 : l;
            h = h2 > h ? h2 : h;
        }
        if ((threadIdx.x & 63) == 0) { mn[a][threadIdx.x >> 6] = l; mx[a][threadIdx.x >> 6] = h; }
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        int a = threadIdx.x;
        unsigned long long l = mn[a][0], h = mx[a][0];
        for (int w = 1; w < 4; ++w) { l = mn[a][w] < l ? mn[a][w] : l; h = mx[a][w] > h ? mx[a][w] : h; }
        atomicMin(&bbox[2 * a], l);
        atomicMax(&bbox[2 * a + 1], h);
    }
}

__global__ void k_pp_keys(int64_t n, Grid g, const double *__restrict__ pos, uint64_t *__restrict__ key,
                          uint32_t *__restrict__ idx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double fx = (pos[i] - g.x0) / g.cell, fy = (pos[n + i] - g.y0) / g.cell, fz = (pos[2 * n + i] - g.z0) / g.cell;
    int cx = min(max((int)floor(fx), 0), g.nx - 1);
    int cy = min(max((int)floor(fy), 0), g.ny - 1);
    int cz = min(max((int)floor(fz), 0), g.nz - 1);
    uint32_t mx = (uint32_t)min(max((int)((fx - cx) * 1024.0), 0), 1023);
    uint32_t my = (uint32_t)min(max((int)((fy - cy) * 1024.0), 0), 1023);
    uint32_t mz = (uint32_t)min(max((int)((fz - cz) * 1024.0), 0), 1023);
    uint64_t cell = ((uint64_t)cz * g.ny + cy) * g.nx + cx;
    key[i] = (cell << 30) | morton3(mx, my, mz);
    idx[i] = (uint32_t)i;
}

// sorted positions (FP64, structure of arrays): the k-th distance can be as small as
// ~1e-2 Mpc/h at distances of ~1e3 Mpc/h, so differences are taken in FP64
__global__ void k_pp_gather(int64_t n, Grid g, const double *__restrict__ pos, const uint64_t *__restrict__ key,
                            const uint32_t *__restrict__ idx, double *__restrict__ sp, uint32_t *__restrict__ cstart,
                            uint32_t *__restrict__ cend) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t j = idx[i];
    uint64_t c = key[i] >> 30;
    sp[i] = pos[j];
    sp[n + i] = pos[n + j];
    sp[2 * n + i] = pos[2 * n + j];
    if (i == 0 || (key[i - 1] >> 30) != c) cstart[c] = (uint32_t)i;
    if (i == n - 1 || (key[i + 1] >> 30) != c) cend[c] = (uint32_t)(i + 1);
}

// particles per coarse cell (cend - cstart, 0 for an empty cell), in place in cend: its exclusive
// prefix sum is the lower-bound array lb[c] = first sorted particle of a cell >= c, so that any run of
// consecutive cells c0 .. c1 - 1 holds exactly the particles [lb[c0], lb[c1])
__global__ void k_pp_cell_counts(int64_t ncells, const uint32_t *__restrict__ cstart, uint32_t *__restrict__ cend) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncells) cend[c] -= cstart[c];
}

// ------------------------------------------------------------ K6 kNN --
constexpr int kKmax = 64;

// The k smallest values seen so far, ascending, in registers: K/16 16-wide vectors indexed only
// by compile-time constants (a runtime index would push the array into scratch memory).  The
// lowest K - k slots hold -inf and never move, so the last slot is always the k-th smallest
// (+inf until k values have arrived).  Insertion shifts the larger entries up by one, branch-free.
// (All values are finite distances or the +-inf sentinels, never NaN.)
typedef float f32x16 __attribute__((ext_vector_type(16)));
template <int K>
struct TopK {
    static_assert(K % 16 == 0, "K must be a multiple of 16");
    f32x16 v[K / 16];
    __device__ void init(int k) {
#pragma unroll
        for (int q = 0; q < K; ++q) v[q >> 4][q & 15] = (q < K - k) ? -__builtin_inff() : __builtin_inff();
    }
    __device__ float at(int q) const { return v[q >> 4][q & 15]; }
    __device__ float kth() const { return at(K - 1); }
    __device__ void push(float x) {
        if (!(x < kth())) return;
        // slot q becomes x clamped to [slot q-1, slot q] (old values, the array being sorted): the
        // median of the three, one v_med3_f32 per slot
#pragma unroll
        for (int q = K - 1; q > 0; --q) v[q >> 4][q & 15] = __builtin_amdgcn_fmed3f(at(q - 1), x, at(q));
        v[0][0] = fminf(v[0][0], x);
    }
};

// first index in [lo, hi) whose key is >= target
__device__ inline uint32_t lower_bound64(const uint64_t *__restrict__ key, uint32_t lo, uint32_t hi, uint64_t target) {
    while (lo < hi) {
        uint32_t mid = lo + ((hi - lo) >> 1);
        if (key[mid] < target) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// The lower bounds of t1 and of t2 in [lo, hi) at once (the Morton block [t1, t2) of a cell): both
// searches are four-way, three probes per step, and step together, so each step's six loads are in
// flight at the same time and the chain of dependent loads is log4 of the range long, not twice its
// log2.
__device__ inline void lower_bound_pair(const uint64_t *__restrict__ key, uint32_t lo, uint32_t hi, uint64_t t1,
                                        uint64_t t2, uint32_t &r1, uint32_t &r2) {
    uint32_t l1 = lo, h1 = hi, l2 = lo, h2 = hi;
    while (h1 - l1 >= 4 || h2 - l2 >= 4) {
        const uint32_t q1 = (h1 - l1) >> 2, q2 = (h2 - l2) >> 2;
        const bool s1 = q1 > 0, s2 = q2 > 0;
        uint64_t a1 = 0, b1 = 0, c1 = 0, a2 = 0, b2 = 0, c2 = 0;
        if (s1) { a1 = key[l1 + q1]; b1 = key[l1 + 2 * q1]; c1 = key[l1 + 3 * q1]; }
        if (s2) { a2 = key[l2 + q2]; b2 = key[l2 + 2 * q2]; c2 = key[l2 + 3 * q2]; }
        if (s1) {
            if (c1 < t1) l1 += 3 * q1 + 1;
            else if (b1 < t1) { h1 = l1 + 3 * q1; l1 += 2 * q1 + 1; }
            else if (a1 < t1) { h1 = l1 + 2 * q1; l1 += q1 + 1; }
            else h1 = l1 + q1;
        }
        if (s2) {
            if (c2 < t2) l2 += 3 * q2 + 1;
            else if (b2 < t2) { h2 = l2 + 3 * q2; l2 += 2 * q2 + 1; }
            else if (a2 < t2) { h2 = l2 + 2 * q2; l2 += q2 + 1; }
            else h2 = l2 + q2;
        }
    }
    r1 = lower_bound64(key, l1, h1, t1);
    r2 = lower_bound64(key, l2, h2, t2);
}

// ----------------------------------- K6b smoothing length from the effective neighbour number --
// h solves N_eff(h) = (4 pi/3) h^3 sum_j W(r_ij, h) = (32/3) sum_j w(r_ij/h) = n_ngb (Sec. 3.4,
// Eq. SPH_kernel), the particle itself included (the standard SPH density sum).  N_eff is continuous,
// non-decreasing and once differentiable in h.  Halley's iteration on h, kept inside a bracket, starts
// from the k-NN distance scaled to the target count; each evaluation sums the kernel and its h-derivatives over
// the particles of every cell within h, on the level whose cells are between h/2 and h wide.
// w(x), g(x) = -x w'(x) and g(x) + x g'(x), which give N_eff and its first two h-derivatives:
// dN/dh = (32/3) sum g / h,  d2N/dh2 = -(32/3) sum (g + x g') / h^2
__device__ inline void wsph_slope(float x, float &w, float &g, float &c) {
    if (x < 0.5f) {
        const float x2 = x * x;
        w = fmaf(6.0f * x2, x - 1.0f, 1.0f);
        g = x2 * fmaf(-18.0f, x, 12.0f);
        c = x2 * fmaf(-72.0f, x, 36.0f);
    } else if (x < 1.0f) {
        const float t = 1.0f - x;
        w = 2.0f * t * t * t;
        g = 6.0f * x * t * t;
        c = 12.0f * x * t * (1.0f - 2.0f * x);
    } else {
        w = 0.0f; g = 0.0f; c = 0.0f;
    }
}

constexpr int kNeffIter = 60;
constexpr double kNeffListMax = 64.0;   // n_ngb up to which the 64-NN list usually holds the root
constexpr int kNeffMaxShell = 4;


// One bracketed Halley step on N_eff(h) - nngb from F = N_eff(h) and its first two h-derivatives:
// updates the bracket [lo, hi] and h, and returns whether the step converged.
__device__ inline bool neff_step(float F, float dF, float d2F, float nngb, float &lo, float &hi, float &h) {
    if (F < nngb) lo = h; else hi = h;
    // Halley's step: third order, since N_eff(h) is twice continuously differentiable (the cubic
    // spline's third derivative jumps where a neighbour crosses h/2, the fourth at h)
    const float Fm = F - nngb, den = 2.0f * dF * dF - Fm * d2F;
    float hn = (dF > 0.0f && den > 0.0f) ? h - 2.0f * Fm * dF / den : 2.0f * h;
    const bool step = hn > lo && hn < hi && hn <= 2.0f * h;
    if (!step) hn = isinf(hi) ? 2.0f * h : 0.5f * (lo + hi);
    // a step below 1e-3 relative: the error left after it is of the order of its cube, ~1e-9,
    // under the FP32 rounding of the sums (stopping at 1e-6 instead costs one more scan for
    // most particles and changes no h by more than that rounding)
    bool conv = step && fabsf(hn - h) <= 1e-3f * h;
    if (!step && !isinf(hi) && hi - lo <= 1e-6f * hi) conv = true;
    h = hn;
    return conv;
}

// One lane per particle, in sorted (cell, Morton) order.  Level-l cells have size cell * 2^(l-10):
// level 10 is the coarse grid, finer levels are aligned Morton blocks inside a coarse cell, and
// coarser ones are blocks of 2^(l-10) coarse cells per axis.  Cells are scanned in Chebyshev shells
// r = 0, 1, 2, ... around the particle's own cell, skipping cells farther than the current k-th
// distance.  After shell r every particle not yet scanned is at least (r + m) cells away, m being
// the particle's distance to its own cell's faces, so the k-th distance is final once it is no
// larger.  The start level makes a cell about the radius that holds k particles at the density of
// the particle's coarse cell; a search that needs more than kShells shells restarts one level up.
constexpr int kShells = 8;
constexpr int kMaxLevel = 20;

// kNeff: after the 64 nearest neighbours (k = K = 64), solve N_eff(h) = nngb from their list (the
// bracketed Halley steps of k_pp_neff, seeded alike from the 32-NN distance times seed_scale).  The
// list holds every particle within h while h does not exceed the 64th distance, so a root at or
// below it is the root; otherwise -(32-NN distance) is written for k_pp_neff to finish.
template <int K, bool kNeff = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(K <= 32 ? 4 : 2)))
k_pp_knn(int64_t n, Grid g, int k, const uint64_t *__restrict__ key, const uint32_t *__restrict__ idx,
         const double *__restrict__ sp, const uint32_t *__restrict__ cstart, const uint32_t *__restrict__ cend,
         float *__restrict__ h_out, int *__restrict__ fail, float nngb = 0.0f, float seed_scale = 0.0f) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t ki = key[i];
    const uint64_t c = ki >> 30;
    const int cx = (int)(c % g.nx), cy = (int)((c / g.nx) % g.ny), cz = (int)(c / ((uint64_t)g.nx * g.ny));
    const double mex = sp[i], mey = sp[n + i], mez = sp[2 * n + i];
    // fine coordinates inside the coarse cell, recovered from the Morton code
    uint32_t m = (uint32_t)(ki & 0x3fffffffu), fx = 0, fy = 0, fz = 0;
    for (int b = 0; b < 10; ++b) {
        fx |= ((m >> (3 * b)) & 1u) << b;
        fy |= ((m >> (3 * b + 1)) & 1u) << b;
        fz |= ((m >> (3 * b + 2)) & 1u) << b;
    }
    const uint32_t occ = cend[c] - cstart[c];
    const double hest = cbrt((double)k / (4.18879 * (double)occ)) * g.cell;   // radius holding k neighbours
    TopK<K> T;
    bool done = false;
    for (int lev = min(max((int)rint(log2(hest / g.cell)) + 10, 0), kMaxLevel); lev <= kMaxLevel && !done; ++lev) {
        // this level's cell grid: size s, the particle's cell (gx, gy, gz), extent (nxl, nyl, nzl)
        const double s = ldexp(g.cell, lev - 10);
        // (int: at most 2^10 times the coarse cells of an axis)
        int gx, gy, gz, nxl, nyl, nzl;
        if (lev <= 10) {
            const int sh = 10 - lev;
            gx = (cx << sh) + (int)(fx >> lev); gy = (cy << sh) + (int)(fy >> lev);
            gz = (cz << sh) + (int)(fz >> lev);
            nxl = g.nx << sh; nyl = g.ny << sh; nzl = g.nz << sh;
        } else {
            const int up = lev - 10;
            gx = cx >> up; gy = cy >> up; gz = cz >> up;
            nxl = (g.nx + (1 << up) - 1) >> up; nyl = (g.ny + (1 << up) - 1) >> up;
            nzl = (g.nz + (1 << up) - 1) >> up;
        }
        // position inside the own cell, in cell units (cell membership came from the same FP64 positions)
        const float ux = fminf(fmaxf((float)((mex - g.x0) / s - (double)gx), 0.0f), 1.0f);
        const float uy = fminf(fmaxf((float)((mey - g.y0) / s - (double)gy), 0.0f), 1.0f);
        const float uz = fminf(fmaxf((float)((mez - g.z0) / s - (double)gz), 0.0f), 1.0f);
        const float mface = fminf(fminf(fminf(ux, 1.0f - ux), fminf(uy, 1.0f - uy)), fminf(uz, 1.0f - uz));
        const float s2 = (float)(s * s);
        // all particles of a contiguous sorted range, eight (then four) at a time: the positions of a
        // group are loaded before its insertions, so their latencies overlap
        auto dist2 = [&](uint32_t j) {
            const float ddx = (float)(sp[j] - mex), ddy = (float)(sp[n + j] - mey), ddz = (float)(sp[2 * n + j] - mez);
            return ddx * ddx + ddy * ddy + ddz * ddz;
        };
        auto scan = [&](uint32_t a0, uint32_t b0) {
            uint32_t j = a0;
            for (; j + 8 <= b0; j += 8) {
                float d2[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) d2[u] = dist2(j + u);
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (j + u != (uint32_t)i) T.push(d2[u]);
            }
            for (; j + 4 <= b0; j += 4) {
                float d2[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) d2[u] = dist2(j + u);
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (j + u != (uint32_t)i) T.push(d2[u]);
            }
            for (; j < b0; ++j)
                if (j != (uint32_t)i) T.push(dist2(j));
        };
        T.init(k);
        for (int r = 0; r <= kShells && !done; ++r) {
            const float kth2 = T.kth();
            for (int dz = -r; dz <= r; ++dz) {
                const int az = gz + dz;
                if (az < 0 || az >= nzl) continue;
                const float ez = dz > 0 ? dz - uz : (dz < 0 ? uz - dz - 1 : 0.0f);
                for (int dy = -r; dy <= r; ++dy) {
                    const int ay = gy + dy;
                    if (ay < 0 || ay >= nyl) continue;
                    const float ey = dy > 0 ? dy - uy : (dy < 0 ? uy - dy - 1 : 0.0f);
                    const bool face = (dz == -r || dz == r || dy == -r || dy == r);
                    const int step = (face || r == 0) ? 1 : 2 * r;
                    for (int dx = -r; dx <= r; dx += step) {
                        const int ax = gx + dx;
                        if (ax < 0 || ax >= nxl) continue;
                        const float ex = dx > 0 ? dx - ux : (dx < 0 ? ux - dx - 1 : 0.0f);
                        // cannot hold a closer particle (the factor absorbs FP32 rounding of both sides)
                        if ((ex * ex + ey * ey + ez * ez) * s2 * 0.999998f >= kth2) continue;
                        if (lev <= 10) {
                            const int sh = 10 - lev;
                            const int ccx = ax >> sh, ccy = ay >> sh, ccz = az >> sh;
                            const uint64_t cc = ((uint64_t)ccz * g.ny + ccy) * g.nx + ccx;
                            uint32_t a0 = cstart[cc], b0 = cend[cc];
                            if (a0 >= b0) continue;
                            if (lev < 10) {
                                const uint32_t lx = (uint32_t)(ax - (ccx << sh)) << lev,
                                               ly = (uint32_t)(ay - (ccy << sh)) << lev,
                                               lz = (uint32_t)(az - (ccz << sh)) << lev;
                                const uint64_t klo = (cc << 30) | morton3(lx, ly, lz);
                                const uint64_t khi = klo + (1ull << (3 * lev));
                                lower_bound_pair(key, a0, b0, klo, khi, a0, b0);
                            }
                            scan(a0, b0);
                        } else {
                            // a row of coarse cells along x is one run of the sorted particles
                            const int up = lev - 10;
                            const int x0 = ax << up, x1 = min((ax + 1) << up, g.nx), y1 = min((ay + 1) << up, g.ny),
                                      z1 = min((az + 1) << up, g.nz);
                            for (int qz = az << up; qz < z1; ++qz)
                                for (int qy = ay << up; qy < y1; ++qy) {
                                    const uint64_t cc = ((uint64_t)qz * g.ny + qy) * g.nx + x0;
                                    scan(cstart[cc], cstart[cc + (x1 - x0)]);
                                }
                        }
                    }
                }
            }
            const float bound = ((float)r + mface) * (float)s * 0.999999f;
            done = T.kth() <= bound * bound;   // +inf (not done) until k neighbours are known
        }
    }
    // a particle too isolated for the largest search gets NaN and raises the failure flag
    if (!done) {
        atomicOr(fail, 1);
        h_out[idx[i]] = __int_as_float(0x7fc00000);
        return;
    }
    if (!kNeff) {
        h_out[idx[i]] = sqrtf(T.kth());
        return;
    }
    // N_eff from the list, the particle itself included (w(0) = 1)
    const float r32 = sqrtf(T.at(31)), rmax2 = T.kth();
    float h = r32 * seed_scale, lo = 0.0f, hi = __builtin_inff();
    bool conv = false, exact = false;   // exact: the last evaluation was at h within the list
    for (int it = 0; it < kNeffIter && !conv; ++it) {
        const float h2 = h * h, ih = 1.0f / h;
        exact = h2 <= rmax2;
        float sw = 1.0f, ss = 0.0f, sc = 0.0f;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const float d2 = T.at(q);
            if (d2 < h2) {
                float wq, gq, cq;
                wsph_slope(sqrtf(d2) * ih, wq, gq, cq);
                sw += wq; ss += gq; sc += cq;
            }
        }
        const float F = (32.0f / 3.0f) * sw, dF = (32.0f / 3.0f) * ss * ih, d2F = -(32.0f / 3.0f) * sc * ih * ih;
        conv = neff_step(F, dF, d2F, nngb, lo, hi, h);
        if (lo * lo >= rmax2) break;   // the root is not below the list's last distance
    }
    // otherwise k_pp_neff finishes from the same seed as without the list (a seed above the root,
    // such as one scaled from N_eff at the 64th distance, makes its first scans wider and slower)
    h_out[idx[i]] = (conv && exact && h * h <= rmax2) ? h : -r32;
}

// With a list, thread t runs the sorted particle list[t] for t < *nlist: the particles the 64-NN
// list could not settle (h_io = -(32-NN distance)), packed so that a wavefront's lanes all work.
// 5 waves per SIMD: 96 VGPRs (104 unconstrained, four waves)
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5)))
k_pp_neff(int64_t n, Grid g, float nngb, float seed_scale,
          const uint64_t *__restrict__ key, const uint32_t *__restrict__ idx,
          const double *__restrict__ sp, const uint32_t *__restrict__ cstart,
          const uint32_t *__restrict__ cend, float *__restrict__ h_io,
          int *__restrict__ fail, const uint32_t *__restrict__ list,
          const uint32_t *__restrict__ nlist) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (list) {
        if (i >= (int64_t)*nlist) return;
        i = list[i];
    } else if (i >= n) {
        return;
    }
    const uint64_t ki = key[i];
    const uint64_t c = ki >> 30;
    const int cx = (int)(c % g.nx), cy = (int)((c / g.nx) % g.ny), cz = (int)(c / ((uint64_t)g.nx * g.ny));
    const double mex = sp[i], mey = sp[n + i], mez = sp[2 * n + i];
    uint32_t m = (uint32_t)(ki & 0x3fffffffu), fx = 0, fy = 0, fz = 0;
    for (int b = 0; b < 10; ++b) {
        fx |= ((m >> (3 * b)) & 1u) << b;
        fy |= ((m >> (3 * b + 1)) & 1u) << b;
        fz |= ((m >> (3 * b + 2)) & 1u) << b;
    }
    const uint32_t oi = idx[i];
    float h = fabsf(h_io[oi]) * seed_scale;
    bool ok = h > 0.0f && isfinite(h);
    float lo = 0.0f, hi = __builtin_inff();
    bool conv = false;
    for (int it = 0; it < kNeffIter && ok && !conv; ++it) {
        // N_eff(h) and dN_eff/dh over the cells within h (cells h/2 to h wide: at most 2 cells out)
        const int lev = min(max((int)ceilf(log2f(h / (float)g.cell)) + 9, 0), kMaxLevel);
        const double s = ldexp(g.cell, lev - 10);
        int gx, gy, gz, nxl, nyl, nzl;
        if (lev <= 10) {
            const int sh = 10 - lev;
            gx = (cx << sh) + (int)(fx >> lev); gy = (cy << sh) + (int)(fy >> lev); gz = (cz << sh) + (int)(fz >> lev);
            nxl = g.nx << sh; nyl = g.ny << sh; nzl = g.nz << sh;
        } else {
            const int up = lev - 10;
            gx = cx >> up; gy = cy >> up; gz = cz >> up;
            nxl = (g.nx + (1 << up) - 1) >> up; nyl = (g.ny + (1 << up) - 1) >> up; nzl = (g.nz + (1 << up) - 1) >> up;
        }
        const float ux = fminf(fmaxf((float)((mex - g.x0) / s - (double)gx), 0.0f), 1.0f);
        const float uy = fminf(fmaxf((float)((mey - g.y0) / s - (double)gy), 0.0f), 1.0f);
        const float uz = fminf(fmaxf((float)((mez - g.z0) / s - (double)gz), 0.0f), 1.0f);
        const float sf = (float)s, h2 = h * h, ih = 1.0f / h;
        const int rmax = (int)ceilf(h / sf);
        if (rmax > kNeffMaxShell) { ok = false; break; }
        float sw = 0.0f, ss = 0.0f, sc = 0.0f;
        auto dist2 = [&](uint32_t j) {
            const float ddx = (float)(sp[j] - mex), ddy = (float)(sp[n + j] - mey), ddz = (float)(sp[2 * n + j] - mez);
            return ddx * ddx + ddy * ddy + ddz * ddz;
        };
        auto add = [&](float r2) {
            if (r2 < h2) {
                float w, gs, cs;
                wsph_slope(sqrtf(r2) * ih, w, gs, cs);
                sw += w; ss += gs; sc += cs;
            }
        };
        // candidates four at a time (positions loaded ahead of the sums, which stay in order)
        auto scan = [&](uint32_t a0, uint32_t b0) {
            uint32_t j = a0;
            for (; j + 4 <= b0; j += 4) {
                float r2[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) r2[u] = dist2(j + u);
#pragma unroll
                for (int u = 0; u < 4; ++u) add(r2[u]);
            }
            for (; j < b0; ++j) add(dist2(j));
        };
        for (int dz = -rmax; dz <= rmax; ++dz) {
            const int az = gz + dz;
            if (az < 0 || az >= nzl) continue;
            const float ez = dz > 0 ? dz - uz : (dz < 0 ? uz - dz - 1 : 0.0f);
            for (int dy = -rmax; dy <= rmax; ++dy) {
                const int ay = gy + dy;
                if (ay < 0 || ay >= nyl) continue;
                const float ey = dy > 0 ? dy - uy : (dy < 0 ? uy - dy - 1 : 0.0f);
                for (int dx = -rmax; dx <= rmax; ++dx) {
                    const int ax = gx + dx;
                    if (ax < 0 || ax >= nxl) continue;
                    const float ex = dx > 0 ? dx - ux : (dx < 0 ? ux - dx - 1 : 0.0f);
                    // no particle of the cell within h (the factor absorbs FP32 rounding)
                    if ((ex * ex + ey * ey + ez * ez) * sf * sf * 0.999998f >= h2) continue;
                    if (lev <= 10) {
                        const int sh = 10 - lev;
                        const int ccx = ax >> sh, ccy = ay >> sh, ccz = az >> sh;
                        const uint64_t cc = ((uint64_t)ccz * g.ny + ccy) * g.nx + ccx;
                        uint32_t a0 = cstart[cc], b0 = cend[cc];
                        if (a0 >= b0) continue;
                        if (lev < 10) {
                            const uint32_t lx = (uint32_t)(ax - (ccx << sh)) << lev, ly = (uint32_t)(ay - (ccy << sh)) << lev,
                                           lz = (uint32_t)(az - (ccz << sh)) << lev;
                            const uint64_t klo = (cc << 30) | morton3(lx, ly, lz);
                            const uint64_t khi = klo + (1ull << (3 * lev));
                            lower_bound_pair(key, a0, b0, klo, khi, a0, b0);
                        }
                        scan(a0, b0);
                    } else {
                        // a row of coarse cells along x is one run of the sorted particles
                        const int up = lev - 10;
                        const int x0 = ax << up, x1 = min((ax + 1) << up, g.nx), y1 = min((ay + 1) << up, g.ny),
                                  z1 = min((az + 1) << up, g.nz);
                        for (int qz = az << up; qz < z1; ++qz)
                            for (int qy = ay << up; qy < y1; ++qy) {
                                const uint64_t cc = ((uint64_t)qz * g.ny + qy) * g.nx + x0;
                                scan(cstart[cc], cstart[cc + (x1 - x0)]);
                            }
                    }
                }
            }
        }
        const float F = (32.0f / 3.0f) * sw, dF = (32.0f / 3.0f) * ss * ih, d2F = -(32.0f / 3.0f) * sc * ih * ih;
        conv = neff_step(F, dF, d2F, nngb, lo, hi, h);
    }
    if (!(ok && conv)) atomicOr(fail, 1);
    h_io[oi] = (ok && conv) ? h : __int_as_float(0x7fc00000);
}

// The particles left to k_pp_neff by the 64-NN list, packed in sorted order: flags (flag[n] = 0),
// their exclusive prefix sum in place, then list[pos[i]] = i (pos[n] is the count).
__global__ void k_pp_fb_flags(int64_t n, const uint32_t *__restrict__ idx, const float *__restrict__ h,
                              uint32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = h[idx[i]] < 0.0f ? 1u : 0u;
    else if (i == n) flag[n] = 0u;
}
__global__ void k_pp_fb_list(int64_t n, const uint32_t *__restrict__ idx, const float *__restrict__ h,
                             const uint32_t *__restrict__ pos, uint32_t *__restrict__ list) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && h[idx[i]] < 0.0f) list[pos[i]] = (uint32_t)i;
}

// ---------------------------------------------------- K7 amplitudes --
struct PPRec {        // per-particle deposit record (40 bytes)
    int32_t ipx, jpx; // particle position in pixel units: integer part ...
    float fpx, fpy;   // ... and fraction, so pixel edges minus position keep their digits
    float ih;         // pixel size / angular smoothing length
    float ay, ab;     // y and b amplitudes (integral of the footprint)
    int32_t i0, j0;   // first pixel column / row of the support square (clipped)
    uint32_t wh;      // width | height << 16 of the clipped support in pixels (0 = no pixels; npix <= 65535)
};

__global__ void __launch_bounds__(256) k_pp_amplitudes(bp_params P, int64_t n, int npix, double pix,
                                                       const float *__restrict__ tx, const float *__restrict__ ty,
                                                       const float *__restrict__ zz, const float *__restrict__ vl,
                                                       const int32_t *__restrict__ hid, const float *__restrict__ ri,
                                                       const float *__restrict__ hcom, double Mp, int64_t nh,
                                                       const double *__restrict__ sol, const int32_t *__restrict__ hst,
                                                       const double *__restrict__ chi_t, const double *__restrict__ tau_t,
                                                       PPRec *__restrict__ rec, uint32_t *__restrict__ wide_flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    PPRec R = {};
    const double z = zz[i];
    const double chi = table_interp(chi_t, z);
    const double DA = chi / (1.0 + z);
    const double u_len = kMpc / P.h, u_mass = kMsun / P.h;
    const double Lpix = DA * pix * u_len;                        // physical pixel size [cm]
    const double ek = exp(-table_interp(tau_t, z));
    const double vc = (double)vl[i] * 1e5 / kC;
    const double mu_e = 2.0 / (1.0 + P.X_H);
    const double Mp_g = Mp * u_mass;
    double ay = 0.0, ab = 0.0;
    const int32_t h = hid[i];
    bool ok = z >= 0.0 && z < kZmax - 0.01;
    if (h < 0) {
        // field gas: Eq. field_b; its tSZ (P_e = n_e k_B T) only when a field temperature is set
        const double Ne = P.field_gas_frac * Mp_g / (mu_e * kMp);
        ay = kSigmaT / kMeC2 * (kKB * P.field_T) * Ne / (Lpix * Lpix);
        ab = kSigmaT * vc * Ne * ek / (Lpix * Lpix);
    } else if (h < nh && !(hst[h] & ~BP_S_MULTI_ROOT)) {
        auto S = [&](int f) { return sol[(int64_t)f * nh + h]; };
        const double r = ri[i];
        const double rs = S(BP_SOL_RS), rv = S(BP_SOL_RVIR), rf = S(BP_SOL_RF), c = S(BP_SOL_C);
        const double x = r / rs;
        const double rho_tot = S(BP_SOL_RHOS) * u_mass / (u_len * u_len * u_len) / (x * (1.0 + x) * (1.0 + x));
        const double V = Mp_g / rho_tot;
        if (r < rf && r > 0.0) {
            double mc = nfw_m(c);
            double ph = (r < rv) ? c / mc * nfw_phi_shape(x) : c * c / ((1.0 + c) * mc) - rv / r;
            double th = 1.0 - S(BP_SOL_A) * ph;
            if (th > 0.0) {
                double th5 = th * th * th * th * th;
                double Rnt = P.alpha_nt * S(BP_SOL_FNT) * pow(r / S(BP_SOL_R500), P.n_nt);
                double Pe = (2.0 * P.X_H + 2.0) / (5.0 * P.X_H + 3.0) * S(BP_SOL_P0) * th5 * th * fmax(0.0, 1.0 - Rnt);
                double ne = S(BP_SOL_RHO0) * th5 / (mu_e * kMp);
                ay = kSigmaT / kMeC2 * Pe * V / (Lpix * Lpix);
                ab = kSigmaT * vc * ek * ne * V / (Lpix * Lpix);
            }
        }
    }
    const double H = (double)hcom[i] / chi;
    ok = ok && H > 0.0 && isfinite(H);
    R.ay = (float)ay; R.ab = (float)ab;
    if (ok && (ay != 0.0 || ab != 0.0)) {
        double px = (double)tx[i] / pix, py = (double)ty[i] / pix;
        double ipx = floor(px), jpy = floor(py);
        R.ipx = (int32_t)fmax(fmin(ipx, 2e9), -2e9); R.jpx = (int32_t)fmax(fmin(jpy, 2e9), -2e9);
        R.fpx = (float)(px - ipx); R.fpy = (float)(py - jpy);
        R.ih = (float)(pix / H);
        double x0 = ((double)tx[i] - H) / pix, x1 = ((double)tx[i] + H) / pix;
        double y0 = ((double)ty[i] - H) / pix, y1 = ((double)ty[i] + H) / pix;
        int i0 = (int)fmax(floor(x0), 0.0), i1 = (int)fmin(floor(x1), (double)(npix - 1));
        int j0 = (int)fmax(floor(y0), 0.0), j1 = (int)fmin(floor(y1), (double)(npix - 1));
        if (i1 >= i0 && j1 >= j0 && x1 >= 0.0 && y1 >= 0.0 && x0 < npix && y0 < npix) {
            R.i0 = i0; R.j0 = j0;
            R.wh = (uint32_t)(i1 - i0 + 1) | ((uint32_t)(j1 - j0 + 1) << 16);
        }
    }
    rec[i] = R;
    if (R.wh) {
        int w = R.wh & 0xffff, hh = R.wh >> 16;
        wide_flag[i] = (w > 24 || hh > 24) ? 1u : 0u;
    } else {
        wide_flag[i] = 2u;   // deposits nothing
    }
}

// ------------------------------------------------------------ K8 deposit --
// Normalised integral of the cubic-spline kernel along one axis (Eq. integrated_kernel),
// evaluated as a left tail: wl(x) = w(x) for x <= 0.  w(x) = 1 - wl(-x) for x > 0.
__device__ inline float wl(float x) {
    if (x <= -1.0f) return 0.0f;
    if (x <= -0.5f) { float t = 1.0f + x, t2 = t * t; return (2.0f / 3.0f) * t2 * t2; }
    float x2 = x * x;
    return (4.0f / 3.0f) * (0.375f + x - 2.0f * x2 * x - 1.5f * x2 * x2);
}
// weight of the cell [a, b] (in units of H, relative to the particle) without cancellation in the tails
__device__ inline float cell_weight(float a, float b) {
    if (a >= 0.0f) return wl(-a) - wl(-b);
    if (b <= 0.0f) return wl(b) - wl(a);
    return 1.0f - wl(a) - wl(-b);
}

constexpr int kPT = 16;   // narrow tiles: 16x16, one wavefront
constexpr int kWT = 64;   // wide tiles: 64x64, one 256-lane workgroup

__global__ void k_pp_count(int64_t n, int ntx_n, int ntx_w, const PPRec *__restrict__ rec,
                           const uint32_t *__restrict__ wide, uint32_t *__restrict__ cnt_n, uint32_t *__restrict__ cnt_w,
                           unsigned long long *__restrict__ totals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t a = 0, b = 0;
    if (i < n) {
        const PPRec R = rec[i];
        if (wide[i] < 2) {
            int w = R.wh & 0xffff, h = R.wh >> 16;
            int T = wide[i] ? kWT : kPT;
            uint32_t nt = (uint32_t)((R.i0 + w - 1) / T - R.i0 / T + 1) * (uint32_t)((R.j0 + h - 1) / T - R.j0 / T + 1);
            if (wide[i]) b = nt; else a = nt;
        }
        cnt_n[i] = a;
        cnt_w[i] = b;
    }
    // per-block totals (64-bit) into totals[2 * block]; k_sum_partials2 adds them up
    __shared__ unsigned long long sa[4], sb[4];
    unsigned long long va = a, vb = b;
    for (int o = 32; o > 0; o >>= 1) { va += __shfl_down(va, o, 64); vb += __shfl_down(vb, o, 64); }
    if ((threadIdx.x & 63) == 0) { sa[threadIdx.x >> 6] = va; sb[threadIdx.x >> 6] = vb; }
    __syncthreads();
    if (threadIdx.x == 0) {
        totals[2 * blockIdx.x] = sa[0] + sa[1] + sa[2] + sa[3];
        totals[2 * blockIdx.x + 1] = sb[0] + sb[1] + sb[2] + sb[3];
    }
    (void)ntx_n; (void)ntx_w;
}

// out[c] = sum over blocks of partial[2 b + c], c = 0, 1 (one workgroup, fixed order per lane)
__global__ void __launch_bounds__(256) k_sum_partials2(int64_t nblocks, const unsigned long long *__restrict__ partial,
                                                       unsigned long long *__restrict__ out) {
    __shared__ unsigned long long s0[256], s1[256];
    unsigned long long a = 0, b = 0;
    for (int64_t i = threadIdx.x; i < nblocks; i += 256) { a += partial[2 * i]; b += partial[2 * i + 1]; }
    s0[threadIdx.x] = a; s1[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) { s0[threadIdx.x] += s0[threadIdx.x + w]; s1[threadIdx.x] += s1[threadIdx.x + w]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[0] = s0[0]; out[1] = s1[0]; }
}

__global__ void k_pp_emit(int64_t n, int ntx_n, int ntx_w, const PPRec *__restrict__ rec, const uint32_t *__restrict__ wide,
                          const uint32_t *__restrict__ off_n, const uint32_t *__restrict__ off_w,
                          uint32_t *__restrict__ kn, uint32_t *__restrict__ vn, uint32_t *__restrict__ kw,
                          uint32_t *__restrict__ vw) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || wide[i] >= 2) return;
    const PPRec R = rec[i];
    const bool W = wide[i] != 0;
    const int T = W ? kWT : kPT, ntx = W ? ntx_w : ntx_n;
    int w = R.wh & 0xffff, h = R.wh >> 16;
    uint32_t o = W ? off_w[i] : off_n[i];
    uint32_t *K = W ? kw : kn, *V = W ? vw : vn;
    for (int ty = R.j0 / T; ty <= (R.j0 + h - 1) / T; ++ty)
        for (int tx = R.i0 / T; tx <= (R.i0 + w - 1) / T; ++tx) {
            K[o] = (uint32_t)(ty * ntx + tx);
            V[o] = (uint32_t)i;
            ++o;
        }
}

__global__ void k_pp_ranges(const uint32_t *__restrict__ keys, int64_t np, uint32_t *__restrict__ ts,
                            uint32_t *__restrict__ te, uint32_t ntiles) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    uint32_t k = keys[i];
    if (k >= ntiles) return;
    if (i == 0 || keys[i - 1] != k) ts[k] = (uint32_t)i;
    if (i == np - 1 || keys[i + 1] != k) te[k] = (uint32_t)(i + 1);
}

__device__ inline void kahan(float &s, float &c, float v) {
    float y = v - c, t = s + y;
    c = (t - s) - y;
    s = t;
}

// narrow particles: one wavefront per 16x16 tile, lane = column (l & 15) x 4 rows
// 7 waves per SIMD: 69 VGPRs (74 unconstrained, six waves)
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7)))
k_pp_deposit_narrow(int npix, double pix, int ntx, uint32_t ntiles,
                    const PPRec *__restrict__ rec, const uint32_t *__restrict__ vals,
                    const uint32_t *__restrict__ ts, const uint32_t *__restrict__ te,
                    float *__restrict__ ymap, float *__restrict__ bmap) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t tile = blockIdx.x * 4 + wave;
    if (tile >= ntiles) return;
    const uint32_t p0 = ts[tile], p1 = te[tile];
    if (p0 >= p1) return;
    const int tx = tile % ntx, ty = tile / ntx;
    const int pi = tx * kPT + (lane & 15), pj0 = ty * kPT + (lane >> 4);
    float ys[4], yc[4], bs[4], bc[4];
    for (int k = 0; k < 4; ++k) {
        int pj = pj0 + 4 * k;
        bool in = pi < npix && pj < npix;
        int64_t id = (int64_t)pj * npix + pi;
        ys[k] = in ? ymap[id] : 0.0f; bs[k] = in ? bmap[id] : 0.0f; yc[k] = 0.0f; bc[k] = 0.0f;
    }
    auto add = [&](const PPRec &R) {
        const int w = R.wh & 0xffff, h = R.wh >> 16;
        if (pi < R.i0 || pi >= R.i0 + w) return;
        // x weight of this lane's column: pixel edges relative to the particle, in units of H
        const float ex = (float)(pi - R.ipx) - R.fpx;
        const float wx = cell_weight(ex * R.ih, (ex + 1.0f) * R.ih);
        for (int k = 0; k < 4; ++k) {
            const int pj = pj0 + 4 * k;
            if (pj < R.j0 || pj >= R.j0 + h) continue;
            const float ey = (float)(pj - R.jpx) - R.fpy;
            const float ay = ey * R.ih, by = (ey + 1.0f) * R.ih;
            const float f = wx * cell_weight(ay, by);
            kahan(ys[k], yc[k], R.ay * f);
            kahan(bs[k], bc[k], R.ab * f);
        }
    };
    // records four at a time: their loads are in flight together, the sums stay in particle order
    uint32_t p = p0;
    for (; p + 4 <= p1; p += 4) {
        PPRec R[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) R[u] = rec[vals[p + u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) add(R[u]);
    }
    for (; p < p1; ++p) add(rec[vals[p]]);
    for (int k = 0; k < 4; ++k) {
        int pj = pj0 + 4 * k;
        if (pi < npix && pj < npix) {
            int64_t id = (int64_t)pj * npix + pi;
            ymap[id] = ys[k]; bmap[id] = bs[k];
        }
    }
}

// wide particles: one 256-lane workgroup per 64x64 tile, 16 pixels per lane (the MFMA output layout).
// Per batch of 8 particles the 64 x- and 64 y-weights of each are staged in LDS.
constexpr int kBatch = 8;
constexpr int kRecWords = sizeof(PPRec) / 4;
typedef float fx4 __attribute__((ext_vector_type(4)));
// 4 waves per SIMD: 121 VGPRs (144 unconstrained, three waves)
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_pp_deposit_wide(int npix, double pix, int ntx, const PPRec *__restrict__ rec,
                  const uint32_t *__restrict__ vals, const uint32_t *__restrict__ ts,
                  const uint32_t *__restrict__ te, float *__restrict__ ymap,
                  float *__restrict__ bmap) {
    // x-weights by particle; y-weights by row (a row's batch contiguous, padded against bank conflicts)
    __shared__ float wxs[kBatch][kWT];
    __shared__ float wys[kWT][kBatch + 1];
    __shared__ float amp[kBatch][2];
    __shared__ uint32_t rsw[kBatch * kRecWords];   // the batch's records
    const uint32_t tile = blockIdx.x;
    const uint32_t p0 = ts[tile], p1 = te[tile];
    if (p0 >= p1) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    // the records of the next batch are fetched (one word per thread) while the current batch runs
    uint32_t pw = 0u;
    auto fetch = [&](uint32_t pb) {
        if (t < kBatch * kRecWords) {
            const uint32_t b = (uint32_t)t / kRecWords, k = (uint32_t)t % kRecWords;
            pw = (pb + b < p1) ? reinterpret_cast<const uint32_t *>(rec + vals[pb + b])[k] : 0u;
        }
    };
    fetch(p0);
    const int tx = tile % ntx, ty = tile / ntx;
    // The batch's update of the tile is the product Wy^T (amp Wx) over its particles, one MFMA
    // (v_mfma_f32_16x16x4_f32, four particles) per 16x16 block and map.  Wavefront w owns the tile
    // rows 16 w .. 16 w + 15; lane l holds the pixels (row 16 w + 4 (l / 16) + j, column 16 bj + l % 16),
    // j, bj < 4, as the MFMA leaves them.
    const int li = lane & 15, lq = lane >> 4;
    const int pi0 = tx * kWT + li, pj0 = ty * kWT + 16 * w + 4 * lq;
    float ys[16], yc[16], bs[16], bc[16];
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * bj + j, pi = pi0 + 16 * bj, pj = pj0 + j;
            const bool in = pi < npix && pj < npix;
            const int64_t id = (int64_t)pj * npix + pi;
            ys[k] = in ? ymap[id] : 0.0f; bs[k] = in ? bmap[id] : 0.0f; yc[k] = 0.0f; bc[k] = 0.0f;
        }
    for (uint32_t pb = p0; pb < p1; pb += kBatch) {
        const int nb = (int)min((uint32_t)kBatch, p1 - pb);
        __syncthreads();
        if (t < kBatch * kRecWords) rsw[t] = pw;
        __syncthreads();
        if (pb + kBatch < p1) fetch(pb + kBatch);
        // stage weights: threads 0..255 cover 8 particles x (64 x-weights or 64 y-weights) in two passes
        for (int q = t; q < kBatch * 2 * kWT; q += 256) {
            int b = q / (2 * kWT), r = q % (2 * kWT);
            float v = 0.0f;
            if (b < nb) {
                PPRec R;
                __builtin_memcpy(&R, &rsw[b * kRecWords], sizeof(PPRec));
                if (r < kWT) {
                    int c = tx * kWT + r;
                    int wd = R.wh & 0xffff;
                    if (c >= R.i0 && c < R.i0 + wd) {
                        float e0 = (float)(c - R.ipx) - R.fpx;
                        v = cell_weight(e0 * R.ih, (e0 + 1.0f) * R.ih);
                    }
                    wxs[b][r] = v;
                } else {
                    int rr = r - kWT, row = ty * kWT + rr;
                    int h = R.wh >> 16;
                    if (row >= R.j0 && row < R.j0 + h) {
                        float e0 = (float)(row - R.jpx) - R.fpy;
                        v = cell_weight(e0 * R.ih, (e0 + 1.0f) * R.ih);
                    }
                    wys[rr][b] = v;
                }
                if (r == 0) { amp[b][0] = R.ay; amp[b][1] = R.ab; }
            } else {                      // unused slot of the last batch: zero weights
                if (r < kWT) wxs[b][r] = 0.0f; else wys[r - kWT][b] = 0.0f;
                if (r == 0) { amp[b][0] = 0.0f; amp[b][1] = 0.0f; }
            }
        }
        __syncthreads();
        // the batch's sums per pixel in FP32 (MFMA), then one compensated update of the pixel's
        // running sum per batch (unused batch slots have zero weights)
        fx4 dy[4], db[4];
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) { dy[bj] = fx4{0.0f, 0.0f, 0.0f, 0.0f}; db[bj] = dy[bj]; }
#pragma unroll
        for (int s4 = 0; s4 < kBatch / 4; ++s4) {
            const int p = 4 * s4 + lq;                    // this lane's particle of the k step
            const float a = wys[16 * w + li][p];          // A[row][p] = Wy[p][row]
            const float ay = amp[p][0], ab = amp[p][1];
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) {
                const float wx = wxs[p][16 * bj + li];    // B[p][col] = amp Wx[p][col]
                dy[bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, ay * wx, dy[bj], 0, 0, 0);
                db[bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, ab * wx, db[bj], 0, 0, 0);
            }
        }
        // rows that no particle of the batch reaches add an exact zero
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                kahan(ys[4 * bj + j], yc[4 * bj + j], dy[bj][j]);
                kahan(bs[4 * bj + j], bc[4 * bj + j], db[bj][j]);
            }
    }
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * bj + j, pi = pi0 + 16 * bj, pj = pj0 + j;
            if (pi < npix && pj < npix) {
                const int64_t id = (int64_t)pj * npix + pi;
                ymap[id] = ys[k]; bmap[id] = bs[k];
            }
        }
}

}  // namespace bp

using namespace bp;

// k-NN distance (n_ngb == 0) or, from it, the effective-neighbour smoothing length (n_ngb > 0)
static int smoothing_length_impl(const bp_params *p, int64_t n, const float *theta_x, const float *theta_y,
                                 const float *z, int32_t k, double n_ngb, double cell, float *h_comoving, void *ws,
                                 size_t ws_bytes, size_t *ws_needed, void *stream) {
    if (check_params(p) || n < 0 || k < 1 || k > kKmax || !ws_needed || !(cell >= 0.0)) return BP_E_ARG;
    if (n == 0) { *ws_needed = 0; return BP_OK; }
    if (!theta_x || !theta_y || !z || !h_comoving) return BP_E_ARG;
    if (n >= 0x7fffffffLL || n <= k) return n <= k ? BP_E_ARG : BP_E_OVERFLOW;
    hipStream_t s = (hipStream_t)stream;
    if (cell == 0.0) cell = 2.0;
    // phase 1: tables, positions, bounding box
    Arena A1(nullptr, 0);
    A1.take<double>(kNZ); A1.take<double>(kNZ);
    A1.take<double>(3 * n);
    A1.take<unsigned long long>(8);
    size_t phase1 = A1.used;
    if (!ws || ws_bytes < phase1) { *ws_needed = phase1 + (size_t)n * 64 + ((size_t)1 << 20); return BP_E_WORKSPACE; }
    Arena A(ws, ws_bytes);
    double *chi_t = A.take<double>(kNZ), *tau_t = A.take<double>(kNZ);
    double *pos = A.take<double>(3 * n);
    unsigned long long *bb = A.take<unsigned long long>(8);
    unsigned long long init[8] = {~0ull, 0ull, ~0ull, 0ull, ~0ull, 0ull, 0ull, 0ull};
    if (hipMemcpyAsync(bb, init, sizeof(init), hipMemcpyHostToDevice, s) != hipSuccess) return BP_E_HIP;
    hipLaunchKernelGGL(k_cosmo_table, dim3((kNZ + 255) / 256), dim3(256), 0, s, *p, gauss_rules(), chi_t, tau_t);
    unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_pp_positions, dim3(blocks < 4096u ? blocks : 4096u), dim3(256), 0, s, n, theta_x, theta_y, z,
                       chi_t, pos, bb,
                       (int *)(bb + 6));
    if (hipGetLastError() != hipSuccess) return BP_E_HIP;
    unsigned long long hb[8];
    if (hipMemcpyAsync(hb, bb, sizeof(hb), hipMemcpyDeviceToHost, s) != hipSuccess) return BP_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return BP_E_HIP;
    if (hb[6]) return BP_E_ARG;   // a redshift outside [0, 16) or a non-finite angle
    auto un = [](unsigned long long u) {
        u = (u & 0x8000000000000000ull) ? (u & 0x7fffffffffffffffull) : ~u;
        double d;
        memcpy(&d, &u, 8);
        return d;
    };
    Grid g;
    g.cell = cell;
    g.x0 = un(hb[0]) - 1e-6 * cell; g.y0 = un(hb[2]) - 1e-6 * cell; g.z0 = un(hb[4]) - 1e-6 * cell;
    double ex = un(hb[1]) - g.x0, ey = un(hb[3]) - g.y0, ez = un(hb[5]) - g.z0;
    g.nx = (int)(ex / cell) + 1; g.ny = (int)(ey / cell) + 1; g.nz = (int)(ez / cell) + 1;
    g.ncells = (int64_t)g.nx * g.ny * g.nz;
    if (g.ncells >= (1LL << 33)) return BP_E_OVERFLOW;
    int cbits = 1;
    while ((1LL << cbits) < g.ncells) ++cbits;
    // phase 2
    size_t need = A.used;
    {
        Arena B(nullptr, 0);
        B.take<uint64_t>(n); B.take<uint64_t>(n); B.take<uint32_t>(n); B.take<uint32_t>(n);
        B.take<double>(3 * n); B.take<uint32_t>(g.ncells + 1); B.take<uint32_t>(g.ncells); B.take<int>(1);
        const size_t rw = radix_ws_bytes(n), sw = scan_ws_bytes(g.ncells), sn = scan_ws_bytes(n + 1);
        need += B.used + std::max(rw, std::max(sw, sn)) + 256;
    }
    if (ws_bytes < need) { *ws_needed = need; return BP_E_WORKSPACE; }
    *ws_needed = need;
    uint64_t *k0 = A.take<uint64_t>(n), *k1 = A.take<uint64_t>(n);
    uint32_t *v0 = A.take<uint32_t>(n), *v1 = A.take<uint32_t>(n);
    double *sp = A.take<double>(3 * n);
    uint32_t *cs = A.take<uint32_t>(g.ncells + 1), *ce = A.take<uint32_t>(g.ncells);
    int *fail = A.take<int>(1);
    void *sws = (char *)ws + A.used;
    prof_begin(BP_PROF_PP_SORT, s);
    hipLaunchKernelGGL(k_pp_keys, dim3(blocks), dim3(256), 0, s, n, g, pos, k0, v0);
    bool in1 = false;
    int e = radix_sort_u64(k0, v0, k1, v1, n, 30 + cbits, sws, s, &in1);
    if (e) return e;
    uint64_t *ks = in1 ? k1 : k0;
    uint32_t *vs = in1 ? v1 : v0;
    if (fill_u32(cs, 0u, g.ncells, s) || fill_u32(ce, 0u, g.ncells, s) || fill_u32((uint32_t *)fail, 0u, 1, s))
        return BP_E_HIP;
    hipLaunchKernelGGL(k_pp_gather, dim3(blocks), dim3(256), 0, s, n, g, pos, ks, vs, sp, cs, ce);
    // cell starts as a lower-bound array (cs[c] for every cell, cs[ncells] = n), cell ends = cs + 1
    hipLaunchKernelGGL(k_pp_cell_counts, dim3((unsigned)((g.ncells + 255) / 256)), dim3(256), 0, s, g.ncells, cs, ce);
    if (hipGetLastError() != hipSuccess) return BP_E_HIP;
    e = scan_exclusive_u32(ce, cs, g.ncells, sws, s);
    if (e) return e;
    if (fill_u32(cs + g.ncells, (uint32_t)n, 1, s)) return BP_E_HIP;
    ce = cs + 1;
    prof_end(BP_PROF_PP_SORT, s);
    prof_begin(BP_PROF_PP_KNN, s);
    // the effective-neighbour length for n_ngb <= 64 starts from the 64-NN list (see k_pp_knn)
    const bool list = n_ngb > 0.0 && n_ngb <= kNeffListMax && n > 64;
    if (list)
        hipLaunchKernelGGL((k_pp_knn<64, true>), dim3(blocks), dim3(256), 0, s, n, g, 64, ks, vs, sp, cs, ce,
                           h_comoving, fail, (float)n_ngb, (float)cbrt(n_ngb / 32.0));
    else if (k <= 16)
        hipLaunchKernelGGL(k_pp_knn<16>, dim3(blocks), dim3(256), 0, s, n, g, (int)k, ks, vs, sp, cs, ce, h_comoving,
                           fail);
    else if (k <= 32)
        hipLaunchKernelGGL(k_pp_knn<32>, dim3(blocks), dim3(256), 0, s, n, g, (int)k, ks, vs, sp, cs, ce, h_comoving,
                           fail);
    else
        hipLaunchKernelGGL(k_pp_knn<64>, dim3(blocks), dim3(256), 0, s, n, g, (int)k, ks, vs, sp, cs, ce, h_comoving,
                           fail);
    prof_end(BP_PROF_PP_KNN, s);
    if (n_ngb > 0.0) {
        // seed: the k-NN distance scaled by (n_ngb / k)^(1/3), the uniform-density ratio
        const float seed = (float)cbrt(n_ngb / (double)k);
        prof_begin(BP_PROF_PP_NEFF, s);
        const uint32_t *fl = nullptr, *nfl = nullptr;
        if (list) {
            // pack the particles left over (the sort's spare buffers: flags and positions in the
            // other key array, the list in the other value array)
            uint32_t *pos = (uint32_t *)(in1 ? k0 : k1), *fb = in1 ? v0 : v1;
            hipLaunchKernelGGL(k_pp_fb_flags, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, s, n, vs,
                               h_comoving, pos);
            if (hipGetLastError() != hipSuccess) return BP_E_HIP;
            e = scan_exclusive_u32(pos, pos, n + 1, sws, s);
            if (e) return e;
            hipLaunchKernelGGL(k_pp_fb_list, dim3(blocks), dim3(256), 0, s, n, vs, h_comoving, pos, fb);
            fl = fb;
            nfl = pos + n;
        }
        hipLaunchKernelGGL(k_pp_neff, dim3(blocks), dim3(256), 0, s, n, g, (float)n_ngb, seed, ks, vs, sp, cs, ce,
                           h_comoving, fail, fl, nfl);
        prof_end(BP_PROF_PP_NEFF, s);
    }
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

extern "C" int bp_pp_smoothing_length(const bp_params *p, int64_t n, const float *theta_x, const float *theta_y,
                                      const float *z, int32_t k, double cell, float *h_comoving, void *ws,
                                      size_t ws_bytes, size_t *ws_needed, void *stream) {
    return smoothing_length_impl(p, n, theta_x, theta_y, z, k, 0.0, cell, h_comoving, ws, ws_bytes, ws_needed,
                                 stream);
}

extern "C" int bp_pp_smoothing_length_eff(const bp_params *p, int64_t n, const float *theta_x, const float *theta_y,
                                          const float *z, double n_ngb, double cell, float *h_comoving, void *ws,
                                          size_t ws_bytes, size_t *ws_needed, void *stream) {
    if (!(n_ngb > 32.0 / 3.0 + 1e-3) || !(n_ngb <= 1024.0)) return BP_E_ARG;
    return smoothing_length_impl(p, n, theta_x, theta_y, z, 32, n_ngb, cell, h_comoving, ws, ws_bytes, ws_needed,
                                 stream);
}

extern "C" int bp_pp_paste_flat(const bp_params *p, int32_t npix, double pix_rad, int64_t n, const float *theta_x,
                                const float *theta_y, const float *z, const float *v_los, const int32_t *halo_id,
                                const float *r_halo, const float *h_comoving, double M_p, int64_t n_halos,
                                const double *sol, const int32_t *status, float *y_map, float *b_map, void *ws,
                                size_t ws_bytes, size_t *ws_needed, void *stream) {
    // npix <= 65535: a particle's clipped footprint width and height share one 32-bit word (16 bits each)
    if (check_params(p) || npix <= 0 || npix > 65535 || !(pix_rad > 0) || n < 0 || !ws_needed || !(M_p > 0) ||
        n_halos < 0)
        return BP_E_ARG;
    if (!y_map || !b_map) return BP_E_ARG;
    if (n == 0) { *ws_needed = 0; return BP_OK; }
    if (!theta_x || !theta_y || !z || !v_los || !halo_id || !r_halo || !h_comoving) return BP_E_ARG;
    if (n_halos > 0 && (!sol || !status)) return BP_E_ARG;
    if (n >= 0x7fffffffLL) return BP_E_OVERFLOW;
    hipStream_t s = (hipStream_t)stream;
    const int ntx_n = (npix + kPT - 1) / kPT, ntx_w = (npix + kWT - 1) / kWT;
    const int64_t nt_n = (int64_t)ntx_n * ntx_n, nt_w = (int64_t)ntx_w * ntx_w;
    Arena A1(nullptr, 0);
    A1.take<double>(kNZ); A1.take<double>(kNZ);
    A1.take<PPRec>(n); A1.take<uint32_t>(n);
    A1.take<uint32_t>(n + 1); A1.take<uint32_t>(n + 1); A1.take<uint32_t>(n + 1); A1.take<uint32_t>(n + 1);
    A1.take<unsigned long long>(2);
    A1.take<unsigned long long>(2 * ((n + 255) / 256));
    size_t phase1 = A1.used + scan_ws_bytes(n + 1);
    if (!ws || ws_bytes < phase1) { *ws_needed = phase1 + 64; return BP_E_WORKSPACE; }
    Arena A(ws, ws_bytes);
    double *chi_t = A.take<double>(kNZ), *tau_t = A.take<double>(kNZ);
    PPRec *rec = A.take<PPRec>(n);
    uint32_t *wide = A.take<uint32_t>(n);
    uint32_t *cn = A.take<uint32_t>(n + 1), *cw = A.take<uint32_t>(n + 1);
    uint32_t *on = A.take<uint32_t>(n + 1), *ow = A.take<uint32_t>(n + 1);
    unsigned long long *tot = A.take<unsigned long long>(2);
    unsigned long long *tot_part = A.take<unsigned long long>(2 * ((n + 255) / 256));
    void *scan_ws = (char *)ws + A.used;
    A.used += scan_ws_bytes(n + 1);
    unsigned blocks = (unsigned)((n + 255) / 256);
    prof_begin(BP_PROF_PP_PLAN, s);
    hipLaunchKernelGGL(k_cosmo_table, dim3((kNZ + 255) / 256), dim3(256), 0, s, *p, gauss_rules(), chi_t, tau_t);
    hipLaunchKernelGGL(k_pp_amplitudes, dim3(blocks), dim3(256), 0, s, *p, n, (int)npix, pix_rad, theta_x, theta_y, z,
                       v_los, halo_id, r_halo, h_comoving, M_p, n_halos, sol, status, chi_t, tau_t, rec, wide);

    if (fill_u32(cn + n, 0u, 1, s) || fill_u32(cw + n, 0u, 1, s)) return BP_E_HIP;
    hipLaunchKernelGGL(k_pp_count, dim3(blocks), dim3(256), 0, s, n, ntx_n, ntx_w, rec, wide, cn, cw, tot_part);
    hipLaunchKernelGGL(k_sum_partials2, dim3(1), dim3(256), 0, s, (int64_t)blocks, tot_part, tot);
    if (hipGetLastError() != hipSuccess) return BP_E_HIP;
    unsigned long long ht[2];
    if (hipMemcpyAsync(ht, tot, sizeof(ht), hipMemcpyDeviceToHost, s) != hipSuccess) return BP_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return BP_E_HIP;
    if (ht[0] >= 0x7fffffffULL || ht[1] >= 0x7fffffffULL) return BP_E_OVERFLOW;
    const int64_t pn = (int64_t)ht[0], pw = (int64_t)ht[1];
    size_t need = A.used;
    {
        Arena B(nullptr, 0);
        for (int q = 0; q < 4; ++q) B.take<uint32_t>(pn);
        for (int q = 0; q < 4; ++q) B.take<uint32_t>(pw);
        B.take<uint32_t>(nt_n); B.take<uint32_t>(nt_n); B.take<uint32_t>(nt_w); B.take<uint32_t>(nt_w);
        need += B.used + radix_ws_bytes(pn > pw ? pn : pw) + 256;
    }
    if (ws_bytes < need) { *ws_needed = need; return BP_E_WORKSPACE; }
    *ws_needed = need;
    uint32_t *kn0 = A.take<uint32_t>(pn), *vn0 = A.take<uint32_t>(pn), *kn1 = A.take<uint32_t>(pn),
             *vn1 = A.take<uint32_t>(pn);
    uint32_t *kw0 = A.take<uint32_t>(pw), *vw0 = A.take<uint32_t>(pw), *kw1 = A.take<uint32_t>(pw),
             *vw1 = A.take<uint32_t>(pw);
    uint32_t *tsn = A.take<uint32_t>(nt_n), *ten = A.take<uint32_t>(nt_n);
    uint32_t *tsw = A.take<uint32_t>(nt_w), *tew = A.take<uint32_t>(nt_w);
    void *sort_ws = (char *)ws + A.used;
    int e = scan_exclusive_u32(cn, on, n + 1, scan_ws, s);
    if (!e) e = scan_exclusive_u32(cw, ow, n + 1, scan_ws, s);
    if (e) return e;
    hipLaunchKernelGGL(k_pp_emit, dim3(blocks), dim3(256), 0, s, n, ntx_n, ntx_w, rec, wide, on, ow, kn0, vn0, kw0,
                       vw0);
    bool in1 = false;
    int bits_n = 1, bits_w = 1;
    while ((1LL << bits_n) < nt_n) ++bits_n;
    while ((1LL << bits_w) < nt_w) ++bits_w;
    e = radix_sort_u32(kn0, vn0, kn1, vn1, pn, bits_n, sort_ws, s, &in1);
    if (e) return e;
    uint32_t *ksn = in1 ? kn1 : kn0, *vsn = in1 ? vn1 : vn0;
    e = radix_sort_u32(kw0, vw0, kw1, vw1, pw, bits_w, sort_ws, s, &in1);
    if (e) return e;
    uint32_t *ksw = in1 ? kw1 : kw0, *vsw = in1 ? vw1 : vw0;
    if (fill_u32(tsn, 0u, nt_n, s) || fill_u32(ten, 0u, nt_n, s) || fill_u32(tsw, 0u, nt_w, s) ||
        fill_u32(tew, 0u, nt_w, s))
        return BP_E_HIP;
    if (pn) hipLaunchKernelGGL(k_pp_ranges, dim3((unsigned)((pn + 255) / 256)), dim3(256), 0, s, ksn, pn, tsn, ten,
                               (uint32_t)nt_n);
    if (pw) hipLaunchKernelGGL(k_pp_ranges, dim3((unsigned)((pw + 255) / 256)), dim3(256), 0, s, ksw, pw, tsw, tew,
                               (uint32_t)nt_w);
    prof_end(BP_PROF_PP_PLAN, s);
    prof_begin(BP_PROF_PP_DEPOSIT, s);
    if (pn) hipLaunchKernelGGL(k_pp_deposit_narrow, dim3((unsigned)((nt_n + 3) / 4)), dim3(256), 0, s, (int)npix,
                               pix_rad, ntx_n, (uint32_t)nt_n, rec, vsn, tsn, ten, y_map, b_map);
    if (pw) hipLaunchKernelGGL(k_pp_deposit_wide, dim3((unsigned)nt_w), dim3(256), 0, s, (int)npix, pix_rad, ntx_w,
                               rec, vsw, tsw, tew, y_map, b_map);
    prof_end(BP_PROF_PP_DEPOSIT, s);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}
