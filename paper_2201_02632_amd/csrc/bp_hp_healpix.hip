// K4: halo-based pasting onto HEALPix RING pixels (the all-sky maps of
// Sec. 5.2 of Osato & Nagai 2022; pixelisation of Gorski et al. 2005).
//
// Tiles are two-dimensional: the rings are taken in bands of eight, and a band
// is cut in longitude into tiles of width 8 * 2 pi / n_max (n_max: the largest
// pixel count among the band's rings), so that a tile holds at most eight
// pixels of each of its rings (exactly eight in the equatorial belt, fewer in
// the shorter rings of a polar band).  Each halo emits one (tile, halo) pair
// per tile that its disc can touch; pairs are stably sorted by tile and one
// wavefront owns a tile (lane = ring of the band * 8 + pixel, y/b sums and
// Kahan compensations in registers).  Per (halo, ring) the colatitude part of
// the haversine, sin^2(dtheta/2), is formed in FP64; per pixel only
// sin^2(dphi/2) is evaluated in FP32:
//   hav = sin^2(dtheta/2) + sin(theta_r) sin(theta_h) sin^2(dphi/2),
//   r_perp = D_A sin(psi) = 2 D_A sqrt(hav (1 - hav)),  psi < pi/2  <=>  hav < 1/2.
#include <hip/hip_runtime.h>
#include <math.h>

#include "bp_device.hpp"
#include "bp_footprint.hpp"
#include "bp_internal.hpp"

namespace bp {

constexpr int kBand = 8;     // rings per band
constexpr int kTw = 8;       // pixels of the longest ring per tile

struct __attribute__((aligned(16))) HpxRec {
    double th, ph, sth;     // halo colatitude, longitude in [0, 2 pi), sin(colatitude)
    float Rt2;              // footprint radius^2 in units of L = D_A theta_pix
    float ra, ra2, rv2;
    float rf, rf2, D, isqD;
    float r2min;
    float eta_lo, eta_ih, om_lo, om_ih, ze_lo, ze_ih;
    float amp_y, amp_b;
    int32_t flags;          // bit0 shell, bit1 zone B, bit2 valid
    float hmax;             // haversine bound used by count and emit (same value in both)
    double ra2d, rf2d;      // r_a^2, r_f^2 in FP64 (edge-annulus recompute)
    double sh2, ch2;        // sin and cos of half the colatitude
    float pad[2];
};
static_assert(sizeof(HpxRec) == 144, "HpxRec size");

struct HpxGeom {
    int64_t N;          // nside
    int32_t nrings;     // 4N - 1
    double pixang;      // sqrt(4 pi / (12 N^2)): the unit length is D_A * pixang
};

// ring i (1-based): number of pixels, first pixel, colatitude and phi shift (in units of the pixel step)
__host__ __device__ inline void ring_info(int64_t N, int64_t i, int64_t *npr, int64_t *off, double *theta,
                                          double *shift) {
    if (i < N) {
        *npr = 4 * i; *off = 2 * i * (i - 1);
        *theta = 2.0 * asin((double)i / (sqrt(6.0) * (double)N));
        *shift = 0.5;
    } else if (i <= 3 * N) {
        *npr = 4 * N; *off = 2 * N * (N - 1) + 4 * N * (i - N);
        *theta = acos((double)(2 * N - i) * 2.0 / (3.0 * (double)N));
        *shift = ((i + N) & 1) ? 1.0 : 0.5;
    } else {
        int64_t k = 4 * N - i;
        *npr = 4 * k; *off = 12 * N * N - 2 * k * (k + 1);
        *theta = kPi - 2.0 * asin((double)k / (sqrt(6.0) * (double)N));
        *shift = 0.5;
    }
}

// real-valued ring coordinate of colatitude t (monotone), for bracketing
__device__ inline double ring_coord(int64_t N, double t) {
    double z = cos(t);
    if (z > 2.0 / 3.0) return sqrt(6.0) * (double)N * sin(0.5 * t);
    if (z < -2.0 / 3.0) return 4.0 * (double)N - sqrt(6.0) * (double)N * cos(0.5 * t);
    return 2.0 * (double)N - 1.5 * (double)N * z;
}

// Per-ring quantities the tile walk and the deposit need, computed once per call (nrings <= 32767).
struct RingRec {
    double th, sth, st2, ct2;   // colatitude, sin(theta), sin(theta/2), cos(theta/2)
    int32_t npr;                // pixels in the ring (<= 4N <= 32768)
    float shift;                // pixel-centre phase: phi_j = (j + 1 - shift) 2 pi / npr, shift 1 or 1/2
    int32_t nmax;               // largest pixel count among the rings of this ring's band
    uint32_t poff;              // first pixel of the ring (< 12 N^2 <= 805,306,368)
};

// largest pixel count among the rings of band b (rings kBand b + 1 .. kBand b + kBand, 1-based)
__device__ inline int32_t band_nmax(int64_t N, int32_t nrings, int b) {
    int64_t m = 0;
    for (int i = kBand * b + 1; i <= min(kBand * b + kBand, nrings); ++i) {
        int64_t npr, off; double th, sh;
        ring_info(N, i, &npr, &off, &th, &sh);
        m = max(m, npr);
    }
    return (int32_t)m;
}

__global__ void k_ring_table(int64_t N, int32_t nrings, RingRec *__restrict__ rt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrings) return;
    int64_t npr, off; double th, sh;
    ring_info(N, i + 1, &npr, &off, &th, &sh);
    RingRec r;
    r.th = th; r.sth = sin(th); r.st2 = sin(0.5 * th); r.ct2 = cos(0.5 * th);
    r.npr = (int32_t)npr; r.shift = (float)sh; r.nmax = band_nmax(N, nrings, i / kBand); r.poff = (uint32_t)off;
    rt[i] = r;
}

// tiles per band: ceil(n_max / 8)
__global__ void k_band_tiles(int64_t N, int32_t nrings, int32_t nbands, uint32_t *__restrict__ ntiles_band) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbands) return;
    ntiles_band[b] = (uint32_t)((band_nmax(N, nrings, b) + kTw - 1) / kTw);
}

// First pixel of tile t in a ring: tile t holds the pixels whose centres satisfy
// 8 t <= (j + 1 - shift) nmax / npr < 8 t + 8, i.e. j >= 8 t npr / nmax - 1 + shift.  Integer
// arithmetic (2 shift is 1 or 2), so that neighbouring tiles agree on every boundary pixel; a tile
// then holds at most ceil(8 npr / nmax) <= 8 pixels of the ring.
__host__ __device__ inline int64_t tile_first_pixel(int64_t t, int64_t npr, int64_t nmax, int s2) {
    const int64_t a = 16 * t * npr + (int64_t)(s2 - 2) * nmax, d = 2 * nmax;
    return a >= 0 ? (a + d - 1) / d : -((-a) / d);
}

// Visit the tiles a halo's disc can touch.  For each ring the disc reaches, the longitudes of
// its pixels that can be members lie within dphi_max of the halo (padded by two pixel steps for
// rounding); per band an interval containing all of these (they are centred on the halo's
// longitude: the band's largest dphi_max with the pad of its coarsest ring, so one arcsine per band)
// is cut into the band's tiles.  f(first, last) is called for runs of consecutive tiles (inclusive)
// in a deterministic order; count and emit use this same routine.  sin((theta_r - theta_h)/2) comes from the half-angle sines and cosines.
template <class F>
__device__ inline void for_each_tile(const HpxGeom &G, const HpxRec &R, const RingRec *__restrict__ rtab,
                                     const uint32_t *__restrict__ btile0, F &&f) {
    const double kTwoPi = 2.0 * kPi;
    double hmax = (double)R.hmax;
    double psi = 2.0 * asin(sqrt(fmin(hmax, 1.0)));
    double tlo = R.th - psi, thi = R.th + psi;
    int64_t ilo = (tlo <= 0.0) ? 1 : (int64_t)floor(ring_coord(G.N, tlo)) - 1;
    int64_t ihi = (thi >= kPi) ? 4 * G.N - 1 : (int64_t)ceil(ring_coord(G.N, thi)) + 1;
    if (ilo < 1) ilo = 1;
    if (ihi > 4 * G.N - 1) ihi = 4 * G.N - 1;
    int band = -1;
    bool any = false, whole = false;
    double qmax = 0.0;      // largest sin^2(dphi/2) bound over the band's rings
    int64_t nprmin = 0;     // fewest pixels of a ring in the band (the widest rounding pad)
    auto flush = [&]() {
        if (!any) return;
        const int nmax = rtab[kBand * band].nmax;
        const int T = (nmax + kTw - 1) / kTw;
        const uint32_t base = btile0[band];
        // one half-width for the whole band: the largest ring's, padded by two steps of its coarsest
        // ring (a superset of the rings' own intervals, which all contain the halo's longitude)
        const double w = whole ? kTwoPi : 2.0 * asin(sqrt(qmax)) + 2.0 * kTwoPi / (double)nprmin;
        const double flo = R.ph - w, fhi = R.ph + w;
        if (!whole && fhi - flo < kTwoPi) {
            const double tpr = (double)nmax / (kTw * kTwoPi);   // tiles per radian
            auto tl = [&](double x) { return (int)fmin(fmax(floor(x * tpr), 0.0), (double)(T - 1)); };
            if (flo >= 0.0 && fhi < kTwoPi) {
                f(base + (uint32_t)tl(flo), base + (uint32_t)tl(fhi));
                return;
            }
            // the interval wraps through phi = 0: [lo1, T) and [0, hi2]
            const int lo1 = tl(flo < 0.0 ? flo + kTwoPi : flo), hi2 = tl(flo < 0.0 ? fhi : fhi - kTwoPi);
            if (hi2 < lo1) {
                f(base, base + (uint32_t)hi2);
                f(base + (uint32_t)lo1, base + (uint32_t)(T - 1));
                return;
            }
        }
        f(base, base + (uint32_t)(T - 1));
    };
    for (int i = (int)ilo; i <= (int)ihi; ++i) {
        const int b = (i - 1) / kBand;
        if (b != band) {
            flush();
            band = b; any = false; whole = false;
        }
        const RingRec &Rg = rtab[i - 1];
        const double sd = Rg.st2 * R.ch2 - Rg.ct2 * R.sh2;
        const double A = sd * sd;
        if (A > hmax) continue;
        const double B = Rg.sth * R.sth;
        const double q = (B > 0.0) ? (hmax - A) / B : 2.0;
        if (q >= 1.0) { whole = true; any = true; continue; }
        if (!any) { qmax = q; nprmin = Rg.npr; }
        else { qmax = fmax(qmax, q); nprmin = min(nprmin, (int64_t)Rg.npr); }
        any = true;
    }
    flush();
}

// Build records and count pairs.  kQ: tables are the surrogate's q-grid (meta holds only PE0, NE0).
template <bool kQ>
__global__ void __launch_bounds__(256) k_hpx_setup(bp_params P, HpxGeom G, int64_t n, const double *__restrict__ th,
                                                   const double *__restrict__ ph, const double *__restrict__ vlos,
                                                   const double *__restrict__ sol, const int32_t *__restrict__ status,
                                                   const float *__restrict__ meta,
                                                   const RingRec *__restrict__ rtab,
                                                   const uint32_t *__restrict__ btile0, HpxRec *__restrict__ rec,
                                                   uint32_t *__restrict__ cnt, unsigned long long *__restrict__ total) {
    __shared__ unsigned long long part[4];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t count = 0;
    if (i < n) {
        HpxRec r = {};
        auto S = [&](int f) { return sol[(int64_t)f * n + i]; };
        auto Mt = [&](int f) { return meta[(int64_t)f * n + i]; };
        double t = th[i], p = ph[i];
        bool ok = !(status[i] & ~BP_S_MULTI_ROOT) && t >= 0.0 && t <= kPi && isfinite(p);
        double DA = S(BP_SOL_DA);
        double L = DA * G.pixang;
        double inv = 1.0 / L;
        double Rt = S(BP_SOL_RT);
        ok = ok && Rt > 0.0 && Rt < DA;
        if (ok) {
            double rv = S(BP_SOL_RVIR) * inv, rf = S(BP_SOL_RF) * inv, ra = fmin(rv, rf), Rtu = Rt * inv;
            p = p - 2.0 * kPi * floor(p / (2.0 * kPi));
            r.th = t; r.ph = p; r.sth = sin(t);
            r.sh2 = sin(0.5 * t); r.ch2 = cos(0.5 * t);
            r.Rt2 = (float)(Rtu * Rtu);
            r.ra = (float)ra; r.ra2 = (float)(ra * ra); r.rv2 = (float)(rv * rv);
            r.rf = (float)rf; r.rf2 = (float)(rf * rf);
            r.ra2d = ra * ra; r.rf2d = rf * rf;
            bool shell = rf > rv;
            double D = shell ? rf * rf - rv * rv : 0.0;
            r.D = (float)D; r.isqD = D > 0.0 ? (float)(1.0 / sqrt(D)) : 0.0f;
            r.r2min = (float)(1e-10 * ra * ra);
            if (!kQ) {
                float elo = Mt(BP_META_ETA_LO), ehi = Mt(BP_META_ETA_HI);
                float olo = Mt(BP_META_OM_LO), ohi = Mt(BP_META_OM_HI);
                float zlo = Mt(BP_META_ZE_LO), zhi = Mt(BP_META_ZE_HI);
                set_zone_grids(r, elo, ehi, olo, ohi, zlo, zhi);
            } else {
                r.eta_lo = (float)Rtu;           // q-grid: R_t in record units and its inverse
                r.eta_ih = (float)(1.0 / Rtu);
            }
            double Lcm = L * kMpc / P.h;
            r.amp_y = (float)(kSigmaT / kMeC2 * (double)Mt(BP_META_PE0) * Lcm);
            r.amp_b = (float)(kSigmaT * (double)Mt(BP_META_NE0) * Lcm * (vlos[i] * 1e5 / kC) * exp(-S(BP_SOL_TAU)));
            r.flags = (shell ? 1 : 0) | ((Rtu > rv) ? 2 : 0) | 4;
            // haversine of the footprint's angular radius (sin psi_max = R_t / D_A), padded for rounding
            double sp = Rt / DA;
            double hav = (sp > 1e-4) ? 0.5 * (1.0 - cos(asin(sp))) : 0.25 * sp * sp * (1.0 + 0.25 * sp * sp);
            r.hmax = (float)(hav * (1.0 + 1e-5) + 1e-30);
            for_each_tile(G, r, rtab, btile0, [&](uint32_t a, uint32_t b) { if (b >= a) count += b - a + 1; });
        }
        rec[i] = r;
        cnt[i] = count;
    }
    unsigned long long v = count;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(total, part[0] + part[1] + part[2] + part[3]);
}

__global__ void __launch_bounds__(256) k_hpx_emit(HpxGeom G, int64_t n, const HpxRec *__restrict__ rec,
                                                  const RingRec *__restrict__ rtab,
                                                  const uint32_t *__restrict__ btile0,
                                                  const uint32_t *__restrict__ off, uint32_t *__restrict__ keys,
                                                  uint32_t *__restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const HpxRec r = rec[i];
    if (!(r.flags & 4)) return;
    uint32_t k = off[i], end = off[i + 1];
    for_each_tile(G, r, rtab, btile0, [&](uint32_t a, uint32_t b) {
        for (uint32_t tile = a; tile <= b && k < end; ++tile) { keys[k] = tile; vals[k] = (uint32_t)i; ++k; }
    });
}

__global__ void k_hpx_ranges(const uint32_t *__restrict__ keys, int64_t np, uint32_t *__restrict__ tstart,
                             uint32_t *__restrict__ tend, uint32_t ntiles) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    uint32_t k = keys[i];
    if (k >= ntiles) return;
    if (i == 0 || keys[i - 1] != k) tstart[k] = (uint32_t)i;
    if (i == np - 1 || keys[i + 1] != k) tend[k] = (uint32_t)(i + 1);
}

// Exact membership next to the edge, in FP64 with the defining expression:
// sin(psi) = |n_pix x n_halo|, n_pix . n_halo > 0, D_A sin(psi) < R_t.
__device__ inline bool hpx_inside_fp64(double tp, double pp, double th, double ph, double DA, double Rt) {
#pragma clang fp contract(off)
    double px = sin(tp) * cos(pp), py = sin(tp) * sin(pp), pz = cos(tp);
    double hx = sin(th) * cos(ph), hy = sin(th) * sin(ph), hz = cos(th);
    double dot = px * hx + py * hy + pz * hz;
    if (!(dot > 0)) return false;
    double cx = py * hz - pz * hy, cy = pz * hx - px * hz, cz = px * hy - py * hx;
    return DA * sqrt(cx * cx + cy * cy + cz * cz) < Rt;
}

template <bool kQ>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_hpx_deposit(HpxGeom G, int64_t n, const HpxRec *__restrict__ rec,
                                                     const float *__restrict__ tables, const uint32_t *__restrict__ vals,
                                                     const uint32_t *__restrict__ tstart, const uint32_t *__restrict__ tend,
                                                     const uint32_t *__restrict__ btile0, int32_t nbands,
                                                     const RingRec *__restrict__ rtab,
                                                     const double *__restrict__ thin, const double *__restrict__ phin,
                                                     const double *__restrict__ sol, float *__restrict__ ymap,
                                                     float *__restrict__ bmap, float *__restrict__ ycomp,
                                                     float *__restrict__ bcomp, uint32_t ntiles) {
    // the tile, its pair range and every halo record are wave-uniform (scalar registers)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const uint32_t tile = blockIdx.x * 4 + wave;
    if (tile >= ntiles) return;
    const uint32_t p0 = tstart[tile], p1 = tend[tile];
    if (p0 >= p1) return;
    // band of this tile: the last band whose first tile is <= tile, by a 64-way search (the lanes probe
    // evenly spaced bands at once; two rounds for the 4,096 bands of N_side 8192 instead of twelve
    // dependent loads).  Invariant: btile0[lo] <= tile < btile0[hi] (btile0[nbands] = all tiles).
    int lo = 0, hi = nbands;
    while (hi - lo > 1) {
        const int step = (hi - lo + 63) / 64;
        const int idx = lo + lane * step;
        const uint64_t m = __ballot(idx < hi && btile0[idx] <= tile);   // bit 0 set: btile0[lo] <= tile
        lo += (63 - __builtin_clzll(m)) * step;
        hi = min(hi, lo + step);
    }
    const int64_t t = tile - btile0[lo];
    // lane = 8 * (ring within the band) + (pixel within the tile's run of that ring)
    const int ring = kBand * lo + 1 + (lane >> 3);
    const RingRec Rr = rtab[min(ring, G.nrings) - 1];
    const int64_t npr = Rr.npr;
    const int s2 = (Rr.shift == 1.0f) ? 2 : 1;
    const int64_t j0 = tile_first_pixel(t, npr, Rr.nmax, s2), j1 = tile_first_pixel(t + 1, npr, Rr.nmax, s2);
    const int64_t jl = j0 + (lane & 7);
    const bool valid = ring <= G.nrings && jl < min(j1, npr);
    const int64_t pix = (int64_t)Rr.poff + jl;
    const double thr = Rr.th, sh = (double)Rr.shift;
    // pixel-centre longitude as the pixelisation defines it: (pi/2)/(npr/4) * (j - shift), j = jl + 1
    const double step = 1.5707963267948966 / (double)(npr / 4);
    const double phj = step * ((double)(jl + 1) - sh);
    const double sthr = Rr.sth, st2 = Rr.st2, ct2 = Rr.ct2;
    const float inv_pix2 = (float)(1.0 / (G.pixang * G.pixang));
    float ys = valid ? ymap[pix] : 0.0f, bs = valid ? bmap[pix] : 0.0f;
    // the compensation carried over from earlier calls, when the caller keeps it
    float yc = (ycomp && valid) ? ycomp[pix] : 0.0f, bc = (bcomp && valid) ? bcomp[pix] : 0.0f;
    for (uint32_t p = p0; p < p1; ++p) {
        const uint32_t h = __builtin_amdgcn_readfirstlane(vals[p]);
        if (h >= (uint32_t)n) continue;
        const HpxRec &R = rec[h];
        const FootRec F = foot_uniform(R);
        // haversine of the angle to the halo: hv = sin^2(dtheta/2) + sin(theta_r) sin(theta_h) sin^2(dphi/2),
        // sin(dtheta/2) from the half-angle sines and cosines of the lane's ring
        const double sd = st2 * R.ch2 - ct2 * R.sh2;
        const float A = (float)(sd * sd), B = (float)(sthr * R.sth);
        // dphi reduced to [-pi, pi] in FP64 before it is rounded to FP32 (a small angle must not be
        // carried as 2 pi minus itself): dphi - 2 pi k with k the nearest integer to dphi / (2 pi), one
        // rounding like the subtraction of 2 pi itself
        double dph = phj - R.ph;
        dph = fma(-2.0 * kPi, rint(dph * (0.5 / kPi)), dph);
        const float xh = (float)(0.5 * dph);
        const float x2 = xh * xh;
        // sin(x) by its odd series below |x| = 0.1 (error < 2e-11 relative), sinf above
        const float s = (fabsf(xh) < 0.1f) ? xh * (1.0f + x2 * (-1.0f / 6.0f + x2 * (1.0f / 120.0f - x2 * (1.0f / 5040.0f))))
                                           : sinf(xh);
        const float hv = A + B * s * s;
        const float r2 = 4.0f * hv * (1.0f - hv) * inv_pix2;
        bool in = (hv < 0.5f) && (r2 < R.Rt2);
        if (fabsf(r2 - R.Rt2) <= 4e-6f * R.Rt2 || fabsf(hv - 0.5f) < 1e-6f) {
            const double DA = sol[(int64_t)BP_SOL_DA * n + h], Rt = sol[(int64_t)BP_SOL_RT * n + h];
            // pixel centre as the pixelisation defines it
            in = hpx_inside_fp64(thr, phj, thin[h], phin[h], DA, Rt);
        }
        if (in && valid) {
            float u2 = R.ra2 - r2, U2 = R.rf2 - r2;
            if ((u2 > 0.0f && u2 < 0.1f * R.ra2) || U2 < 0.1f * R.rf2) {
                // next to r_a (inside) or r_f: recompute the haversine in FP64 so the square root of the
                // small difference keeps its digits; in zone B only the sign of u^2 is used
                double sp = sin(0.5 * (phj - R.ph));
                double hvd = sd * sd + sthr * R.sth * sp * sp;
                double r2d = 4.0 * hvd * (1.0 - hvd) / (G.pixang * G.pixang);
                u2 = (float)(R.ra2d - r2d);
                U2 = (float)(R.rf2d - r2d);
            }
            float vp, vn;
            if (kQ) footprint_value_q(R, tables + (int64_t)h * 2 * BP_MLP_NQ, r2, U2, &vp, &vn);
            else footprint_value(F, tables + (int64_t)h * BP_TAB_STRIDE, r2, u2, U2, &vp, &vn);
            kahan_add(ys, yc, R.amp_y * vp);
            kahan_add(bs, bc, R.amp_b * vn);
        }
    }
    if (valid) {
        ymap[pix] = ys; bmap[pix] = bs;
        if (ycomp) ycomp[pix] = yc;
        if (bcomp) bcomp[pix] = bc;
    }
}

}  // namespace bp

using namespace bp;

template <bool kQ>
static int paste_healpix_impl(const bp_params *p, int64_t nside, int64_t n, const double *theta, const double *phi,
                              const double *v_los, const double *sol, const int32_t *status, const float *tables,
                              const float *meta, float *y_map, float *b_map, float *y_comp, float *b_comp, void *ws,
                              size_t ws_bytes, size_t *ws_needed, void *stream, hipStream_t plan_stream = nullptr,
                              hipEvent_t plan_done = nullptr) {
    if (check_params(p) || nside < 1 || nside > 8192 || n < 0 || !ws_needed) return BP_E_ARG;
    if (n > 0 && (!theta || !phi || !v_los || !sol || !status || !tables || !meta)) return BP_E_ARG;
    if (!y_map || !b_map) return BP_E_ARG;
    if (n >= 0x7fffffffLL) return BP_E_OVERFLOW;
    if (n == 0) { *ws_needed = 0; return BP_OK; }
    hipStream_t s = (hipStream_t)stream;
    // set-up and plan run on plan_stream when one is given (its own dependencies set by the caller),
    // the deposit on stream after plan_done
    hipStream_t sp = plan_stream ? plan_stream : s;
    HpxGeom G;
    G.N = nside;
    G.nrings = (int32_t)(4 * nside - 1);
    G.pixang = sqrt(4.0 * kPi / (12.0 * (double)nside * (double)nside));
    const int32_t nbands = (G.nrings + kBand - 1) / kBand;
    Arena A1(nullptr, 0);
    A1.take<HpxRec>(n);
    A1.take<uint32_t>(n + 1);
    A1.take<uint32_t>(n + 1);
    A1.take<unsigned long long>(1);
    A1.take<uint32_t>(nbands + 1);
    A1.take<uint32_t>(nbands + 1);
    A1.take<RingRec>(G.nrings);
    size_t phase1 = A1.used + scan_ws_bytes(n + 1) + scan_ws_bytes(nbands + 1);
    if (ws_bytes < phase1 || !ws) { *ws_needed = phase1 + 64; return BP_E_WORKSPACE; }
    Arena A(ws, ws_bytes);
    HpxRec *rec = A.take<HpxRec>(n);
    uint32_t *cnt = A.take<uint32_t>(n + 1);
    uint32_t *off = A.take<uint32_t>(n + 1);
    unsigned long long *total = A.take<unsigned long long>(1);
    uint32_t *btiles = A.take<uint32_t>(nbands + 1);
    uint32_t *btile0 = A.take<uint32_t>(nbands + 1);
    RingRec *rtab = A.take<RingRec>(G.nrings);
    void *scan_ws = (char *)ws + A.used;
    A.used += scan_ws_bytes(n + 1) + scan_ws_bytes(nbands + 1);
    // tiles per band and their prefix (the total lands in btile0[nbands])
    if (fill_u32(btiles + nbands, 0u, 1, sp)) return BP_E_HIP;
    hipLaunchKernelGGL(k_band_tiles, dim3((nbands + 255) / 256), dim3(256), 0, sp, G.N, G.nrings, nbands, btiles);
    if (hipGetLastError() != hipSuccess) return BP_E_HIP;
    int e = scan_exclusive_u32(btiles, btile0, nbands + 1, scan_ws, sp);
    if (e) return e;
    hipLaunchKernelGGL(k_ring_table, dim3((G.nrings + 255) / 256), dim3(256), 0, sp, G.N, G.nrings, rtab);
    if (fill_u32((uint32_t *)total, 0u, 2, sp)) return BP_E_HIP;   // a fill kernel rather than a memset node
    if (fill_u32(cnt + n, 0u, 1, sp)) return BP_E_HIP;
    unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_hpx_setup<kQ>, dim3(blocks), dim3(256), 0, sp, *p, G, n, theta, phi, v_los, sol, status,
                       meta, rtab, btile0, rec, cnt, total);
    if (hipGetLastError() != hipSuccess) return BP_E_HIP;
    unsigned long long np64 = 0;
    uint32_t ntiles32 = 0;
    if (hipMemcpyAsync(&np64, total, sizeof(np64), hipMemcpyDeviceToHost, sp) != hipSuccess) return BP_E_HIP;
    if (hipMemcpyAsync(&ntiles32, btile0 + nbands, sizeof(uint32_t), hipMemcpyDeviceToHost, sp) != hipSuccess)
        return BP_E_HIP;
    if (hipStreamSynchronize(sp) != hipSuccess) return BP_E_HIP;
    if (np64 >= 0x7fffffffULL) return BP_E_OVERFLOW;
    const int64_t np = (int64_t)np64, ntiles = ntiles32;
    size_t need = A.used;
    {
        Arena B(nullptr, 0);
        for (int q = 0; q < 4; ++q) B.take<uint32_t>(np);
        B.take<uint32_t>(ntiles);
        B.take<uint32_t>(ntiles);
        need += B.used + radix_ws_bytes(np) + 256;
    }
    if (ws_bytes < need) { *ws_needed = need; return BP_E_WORKSPACE; }
    *ws_needed = need;
    if (np == 0) return BP_OK;
    uint32_t *k0 = A.take<uint32_t>(np), *v0 = A.take<uint32_t>(np);
    uint32_t *k1 = A.take<uint32_t>(np), *v1 = A.take<uint32_t>(np);
    uint32_t *tst = A.take<uint32_t>(ntiles), *ten = A.take<uint32_t>(ntiles);
    void *sort_ws = (char *)ws + A.used;
    prof_begin(BP_PROF_HPX_PLAN, sp);
    e = scan_exclusive_u32(cnt, off, n + 1, scan_ws, sp);
    if (e) return e;
    hipLaunchKernelGGL(k_hpx_emit, dim3(blocks), dim3(256), 0, sp, G, n, rec, rtab, btile0, off, k0, v0);
    if (hipGetLastError() != hipSuccess) return BP_E_HIP;
    int bits = 1;
    while ((1LL << bits) < ntiles) ++bits;
    bool in1 = false;
    e = radix_sort_u32(k0, v0, k1, v1, np, bits, sort_ws, sp, &in1);
    if (e) return e;
    uint32_t *ks = in1 ? k1 : k0, *vs = in1 ? v1 : v0;
    if (fill_u32(tst, 0u, ntiles, sp) || fill_u32(ten, 0u, ntiles, sp)) return BP_E_HIP;
    hipLaunchKernelGGL(k_hpx_ranges, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, sp, ks, np, tst, ten,
                       (uint32_t)ntiles);
    if (hipGetLastError() != hipSuccess) return BP_E_HIP;
    prof_end(BP_PROF_HPX_PLAN, sp);
    if (sp != s) {
        if (hipEventRecord(plan_done, sp) != hipSuccess || hipStreamWaitEvent(s, plan_done, 0) != hipSuccess)
            return BP_E_HIP;
    }
    prof_begin(kQ ? BP_PROF_HPXQ_DEPOSIT : BP_PROF_HPX_DEPOSIT, s);
    hipLaunchKernelGGL(k_hpx_deposit<kQ>, dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, s, G, n, rec, tables, vs,
                       tst, ten, btile0, nbands, rtab, theta, phi, sol, y_map, b_map, y_comp, b_comp,
                       (uint32_t)ntiles);
    prof_end(kQ ? BP_PROF_HPXQ_DEPOSIT : BP_PROF_HPX_DEPOSIT, s);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

extern "C" int bp_hp_paste_healpix(const bp_params *p, int64_t nside, int64_t n, const double *theta,
                                   const double *phi, const double *v_los, const double *sol, const int32_t *status,
                                   const float *tables, const float *meta, float *y_map, float *b_map, float *y_comp,
                                   float *b_comp, void *ws, size_t ws_bytes, size_t *ws_needed, void *stream) {
    return paste_healpix_impl<false>(p, nside, n, theta, phi, v_los, sol, status, tables, meta, y_map, b_map, y_comp,
                                     b_comp, ws, ws_bytes, ws_needed, stream);
}

extern "C" int bp_hp_paste_healpix_q(const bp_params *p, int64_t nside, int64_t n, const double *theta,
                                     const double *phi, const double *v_los, const double *sol,
                                     const int32_t *status, const float *qtables, const float *meta, float *y_map,
                                     float *b_map, float *y_comp, float *b_comp, void *ws, size_t ws_bytes,
                                     size_t *ws_needed, void *stream) {
    return paste_healpix_impl<true>(p, nside, n, theta, phi, v_los, sol, status, qtables, meta, y_map, b_map, y_comp,
                                    b_comp, ws, ws_bytes, ws_needed, stream);
}

int bp::paste_healpix_q_planned(const bp_params *p, int64_t nside, int64_t n, const double *theta, const double *phi,
                                const double *v_los, const double *sol, const int32_t *status, const float *qtables,
                                const float *meta, float *y_map, float *b_map, float *y_comp, float *b_comp, void *ws,
                                size_t ws_bytes, size_t *ws_needed, hipStream_t stream, hipStream_t plan_stream,
                                hipEvent_t plan_done) {
    return paste_healpix_impl<true>(p, nside, n, theta, phi, v_los, sol, status, qtables, meta, y_map, b_map, y_comp,
                                    b_comp, ws, ws_bytes, ws_needed, stream, plan_stream, plan_done);
}

// ---------------------------------------------------------- one-call pipeline --
extern "C" int bp_hp_healpix_pipeline(const bp_params *p, int64_t nside, int64_t n, const double *M, const double *c,
                                      const double *z, const double *theta, const double *phi, const double *v_los,
                                      double *sol, int32_t *status, float *tables, float *meta, float *y_map,
                                      float *b_map, float *y_comp, float *b_comp, void *ws, size_t ws_bytes,
                                      size_t *ws_needed, void *stream) {
    if (check_params(p) || nside < 1 || nside > 8192 || n < 0 || !ws_needed) return BP_E_ARG;
    if (!y_map || !b_map) return BP_E_ARG;
    if (n > 0 && (!M || !c || !z || !theta || !phi || !v_los || !sol || !status || !tables || !meta)) return BP_E_ARG;
    if (n >= 0x7fffffffLL) return BP_E_OVERFLOW;
    if (n == 0) { *ws_needed = 0; return BP_OK; }
    SideStream *S = nullptr;
    int e = side_stream_for_current_device(&S);
    if (e) return e;
    std::lock_guard<std::mutex> lock(S->mu);
    hipStream_t s = (hipStream_t)stream;
    if ((e = bp_icm_solve(p, n, M, c, z, sol, status, stream))) return e;
    // the quadratures stay queued on `stream`; the paste's set-up needs only the solve and meta
    if ((e = profile_tables_launch(p, n, sol, status, tables, meta, s, S->meta_ready))) return e;
    if (hipStreamWaitEvent(S->s, S->meta_ready, 0) != hipSuccess) return BP_E_HIP;
    e = paste_healpix_impl<false>(p, nside, n, theta, phi, v_los, sol, status, tables, meta, y_map, b_map, y_comp,
                                  b_comp, ws, ws_bytes, ws_needed, stream, S->s, S->plan_done);
    return e ? join_side(S, s, e) : BP_OK;
}
