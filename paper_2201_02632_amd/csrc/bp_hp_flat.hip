// K3: halo-based pasting onto a flat-sky map (Sec. 3.3 of Osato & Nagai 2022).
//
// The map is cut into 16x16-pixel tiles.  Every halo emits one (tile, halo)
// pair per tile that its footprint disc touches; the pairs are stably sorted
// by tile, so each tile's list is in catalogue order.  One wavefront owns one
// tile: lane l holds one pixel of each 8x8 quadrant (column l%8, row l/8) with
// its y and b sums and Kahan compensations in registers, walks the tile's halo
// list (halo records are wave-uniform scalar loads), and writes the tile back
// once.  A quadrant the disc misses costs only the membership test: its
// profile evaluation is branched over for the whole wave.  No atomics touch
// the maps, and the summation order is fixed.
#include <hip/hip_runtime.h>
#include <math.h>

#include <mutex>

#include "bp_device.hpp"
#include "bp_internal.hpp"
#include "bp_footprint.hpp"

namespace bp {

constexpr int kTile = 16;

// Per-halo paste record in pixel units (176 bytes; read by each wave as scalar loads).
struct __attribute__((aligned(16))) FlatRec {
    int32_t cxi, cyi;       // integer part of the centre in pixel units
    float hx, hy;           // 0.5 minus the fractional part: pixel (i, j) sits at (i - cxi + hx, j - cyi + hy)
    float Rt2;              // footprint radius^2 [px^2]
    float Rt2_band;         // 4e-6 Rt2: FP32 distances this close to the edge are re-decided in FP64
    float ra, ra2;          // r_a = min(r_vir, r_f), r_a^2
    float rf, rf2, D, isqD; // r_f, r_f^2, r_f^2 - r_vir^2, 1/sqrt(D) (0 without a shell)
    float ra2_edge, rf2_edge;  // 0.1 r_a^2, 0.1 r_f^2: below these u^2 and U^2 are formed in FP64
    float r2min;            // clamp of r_perp^2 at the centre
    float eta_lo, eta_ih;   // zone A grid start and 1/step (log2 units)
    float om_lo, om_ih;     // zone S
    float ze_lo, ze_ih;     // zone B
    float amp_y, amp_b;     // sigma_T/(m_e c^2) P_e0 L_pix ; sigma_T n_e0 L_pix (v/c) e^-tau
    int32_t flags;          // bit0 shell (r_f > r_vir), bit1 zone B (R_t > r_vir), bit2 valid
    float Rt_emit;          // footprint radius used by both the pair count and the emit pass
    float pad[3];
    double cxd, cyd;        // fractional centre in FP64 (edge-annulus recompute)
    double ra2d, rf2d;      // r_a^2, r_f^2 in FP64
    double thx, thy;        // centre [rad] and, below, D_A and R_t [Mpc/h]: the exact membership test
    double DA, Rt;
};
static_assert(sizeof(FlatRec) == 176, "FlatRec size");

// The first 96 bytes of a record: every field a pair needs outside the FP64 edge re-tests.
struct FlatHead {
    int32_t cxi, cyi;
    float hx, hy, Rt2, Rt2_band, ra, ra2, rf, rf2, D, isqD, ra2_edge, rf2_edge, r2min;
    float eta_lo, eta_ih, om_lo, om_ih, ze_lo, ze_ih, amp_y, amp_b;
    int32_t flags;
};
static_assert(sizeof(FlatHead) == 96 && offsetof(FlatRec, flags) == 92, "FlatHead mirrors FlatRec");

// Load a record head into scalar registers in one batch.  The empty asm statement takes the 24
// words as opaque inputs and outputs, so the compiler issues all their loads before one wait and
// keeps the values, instead of splitting the loads around register reuse and reloading fields
// later (each split costs a scalar-memory round trip per pair).
__device__ inline FlatHead load_head(const FlatRec *rec, uint32_t h) {
    const uint32_t *p = reinterpret_cast<const uint32_t *>(rec + h);
    uint32_t w[24];
#pragma unroll
    for (int j = 0; j < 24; ++j) w[j] = __builtin_amdgcn_readfirstlane(p[j]);
    asm volatile("" : "+s"(w[0]), "+s"(w[1]), "+s"(w[2]), "+s"(w[3]), "+s"(w[4]), "+s"(w[5]), "+s"(w[6]),
                 "+s"(w[7]), "+s"(w[8]), "+s"(w[9]), "+s"(w[10]), "+s"(w[11]));
    asm volatile("" : "+s"(w[12]), "+s"(w[13]), "+s"(w[14]), "+s"(w[15]), "+s"(w[16]), "+s"(w[17]),
                 "+s"(w[18]), "+s"(w[19]), "+s"(w[20]), "+s"(w[21]), "+s"(w[22]), "+s"(w[23]));
    FlatHead H;
    __builtin_memcpy(&H, w, sizeof(H));
    return H;
}

__device__ inline void tile_row_range(double cx, double cy, double Rt, int ty, int ntx, int npix, int *tx0, int *tx1) {
    // pixel rows of this tile: centres y in [16 ty + 0.5, 16 ty + 15.5]
    double ylo = kTile * ty + 0.5, yhi = kTile * ty + kTile - 0.5;
    double yc = fmin(fmax(cy, ylo), yhi);
    double dy = fabs(yc - cy);
    double R = Rt + 1.0;  // one-pixel margin: the deposit decides membership exactly
    if (dy > R) { *tx0 = 1; *tx1 = 0; return; }
    double hw = sqrt(R * R - dy * dy);
    double xl = cx - hw - 0.5, xh = cx + hw - 0.5;  // pixel index range
    int il = (int)fmax(floor(xl), 0.0), ih = (int)fmin(floor(xh) + 1.0, (double)(npix - 1));
    if (il > ih) { *tx0 = 1; *tx1 = 0; return; }
    *tx0 = il / kTile;
    *tx1 = ih / kTile;
    (void)ntx;
}

struct FlatGeom {
    int npix, ntx;
    double pix;
};

// Build records and count pairs.  kQ: tables are the surrogate's q-grid (meta holds only PE0, NE0).
template <bool kQ>
__global__ void __launch_bounds__(256) k_flat_setup(bp_params P, FlatGeom Gm, int64_t n, const double *__restrict__ thx,
                                                    const double *__restrict__ thy, const double *__restrict__ vlos,
                                                    const double *__restrict__ sol, const int32_t *__restrict__ status,
                                                    const float *__restrict__ meta, FlatRec *__restrict__ rec,
                                                    uint32_t *__restrict__ cnt, unsigned long long *__restrict__ total) {
    __shared__ unsigned long long part[4];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t count = 0;
    if (i < n) {
        FlatRec r = {};
        auto S = [&](int f) { return sol[(int64_t)f * n + i]; };
        auto Mt = [&](int f) { return meta[(int64_t)f * n + i]; };
        bool ok = !(status[i] & ~BP_S_MULTI_ROOT);
        double DA = S(BP_SOL_DA);
        double Lpix = DA * Gm.pix;       // physical Mpc/h per pixel
        double inv = 1.0 / Lpix;
        double cx = thx[i] / Gm.pix, cy = thy[i] / Gm.pix;
        double Rt = S(BP_SOL_RT) * inv;
        ok = ok && isfinite(cx) && isfinite(cy) && Rt > 0.0 && isfinite(Rt);
        // drop halos whose disc misses the map entirely
        ok = ok && (cx + Rt > 0.0) && (cy + Rt > 0.0) && (cx - Rt < Gm.npix) && (cy - Rt < Gm.npix);
        if (ok) {
            double rv = S(BP_SOL_RVIR) * inv, rf = S(BP_SOL_RF) * inv;
            double ra = fmin(rv, rf);
            double cxf = floor(cx), cyf = floor(cy);
            r.cxi = (int32_t)cxf; r.cyi = (int32_t)cyf;
            r.hx = 0.5f - (float)(cx - cxf); r.hy = 0.5f - (float)(cy - cyf);
            r.Rt2 = (float)(Rt * Rt);
            r.Rt2_band = 4e-6f * r.Rt2;
            r.ra = (float)ra; r.ra2 = (float)(ra * ra);
            r.rf = (float)rf; r.rf2 = (float)(rf * rf);
            r.ra2_edge = 0.1f * r.ra2; r.rf2_edge = 0.1f * r.rf2;
            r.cxd = cx - cxf; r.cyd = cy - cyf;
            r.ra2d = ra * ra; r.rf2d = rf * rf;
            r.thx = thx[i]; r.thy = thy[i];
            r.DA = DA; r.Rt = S(BP_SOL_RT);
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
                r.eta_lo = (float)Rt;       // q-grid: R_t in pixels and its inverse
                r.eta_ih = (float)(1.0 / Rt);
            }
            double Lcm = Lpix * kMpc / P.h;
            r.amp_y = (float)(kSigmaT / kMeC2 * (double)Mt(BP_META_PE0) * Lcm);
            r.amp_b = (float)(kSigmaT * (double)Mt(BP_META_NE0) * Lcm * (vlos[i] * 1e5 / kC) * exp(-S(BP_SOL_TAU)));
            bool zoneB = Rt > rv;
            r.flags = (shell ? 1 : 0) | (zoneB ? 2 : 0) | 4;
            // count tiles touched; the emit pass repeats this loop with the same (float) radius
            r.Rt_emit = (float)Rt;
            double Rtd = (double)r.Rt_emit;
            int ty0 = (int)fmax(floor((cy - Rtd - 1.5) / kTile), 0.0);
            int ty1 = (int)fmin(floor((cy + Rtd + 0.5) / kTile), (double)(Gm.ntx - 1));
            for (int ty = ty0; ty <= ty1; ++ty) {
                int a, b;
                tile_row_range(cx, cy, Rtd, ty, Gm.ntx, Gm.npix, &a, &b);
                if (b >= a) count += (uint32_t)(b - a + 1);
            }
        }
        rec[i] = r;
        cnt[i] = count;
    }
    // block total of pair counts, in 64 bits, for the overflow check
    unsigned long long v = count;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(total, part[0] + part[1] + part[2] + part[3]);
}

__global__ void __launch_bounds__(256) k_flat_emit(FlatGeom Gm, int64_t n, const double *__restrict__ thx,
                                                   const double *__restrict__ thy, const FlatRec *__restrict__ rec,
                                                   const uint32_t *__restrict__ off, uint32_t *__restrict__ keys,
                                                   uint32_t *__restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !(rec[i].flags & 4)) return;
    double cx = thx[i] / Gm.pix, cy = thy[i] / Gm.pix;
    uint32_t o = off[i], end = off[i + 1];
    uint32_t k = o;
    double Rtd = (double)rec[i].Rt_emit;
    int ty0 = (int)fmax(floor((cy - Rtd - 1.5) / kTile), 0.0);
    int ty1 = (int)fmin(floor((cy + Rtd + 0.5) / kTile), (double)(Gm.ntx - 1));
    for (int ty = ty0; ty <= ty1 && k < end; ++ty) {
        int a, b;
        tile_row_range(cx, cy, Rtd, ty, Gm.ntx, Gm.npix, &a, &b);
        for (int tx = a; tx <= b && k < end; ++tx) {
            keys[k] = (uint32_t)(ty * Gm.ntx + tx);
            vals[k] = (uint32_t)i;
            ++k;
        }
    }
}

__global__ void k_tile_ranges(const uint32_t *__restrict__ keys, int64_t np, uint32_t *__restrict__ tstart,
                              uint32_t *__restrict__ tend, uint32_t ntiles) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    uint32_t k = keys[i];
    if (k >= ntiles) return;
    if (i == 0 || keys[i - 1] != k) tstart[k] = (uint32_t)i;
    if (i == np - 1 || keys[i + 1] != k) tend[k] = (uint32_t)(i + 1);
}

// Membership of pixel (i, j): FP32 test, re-decided in FP64 next to the edge
// with the same expression the definition uses: D_A |theta_pix - theta_h| < R_t.
__device__ inline bool inside_fp64(int i, int j, double pix, double thx, double thy, double DA, double Rt) {
#pragma clang fp contract(off)
    double dx = (i + 0.5) * pix - thx, dy = (j + 0.5) * pix - thy;
    double rp = DA * sqrt(dx * dx + dy * dy);
    return rp < Rt;
}

template <bool kQ>
__global__ void __launch_bounds__(256) k_flat_deposit(FlatGeom Gm, int64_t n, const FlatRec *__restrict__ rec,
                                                      const float *__restrict__ tables, const uint32_t *__restrict__ vals,
                                                      const uint32_t *__restrict__ tstart, const uint32_t *__restrict__ tend,
                                                      float *__restrict__ ymap, float *__restrict__ bmap,
                                                      float *__restrict__ ycomp, float *__restrict__ bcomp, int ntiles) {
    // the tile, its pair range and every halo record are wave-uniform (scalar registers)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + wave;
    if (tile >= ntiles) return;
    const uint32_t p0 = tstart[tile], p1 = tend[tile];
    if (p0 >= p1) return;
    const int tx = tile % Gm.ntx, ty = tile / Gm.ntx;
    // pass q covers the 8x8 quadrant (q & 1, q >> 1) of the tile; lane l holds its pixel (l % 8, l / 8)
    const int X0 = tx * kTile, Y0 = ty * kTile;
    const int li = lane & 7, lj = lane >> 3;
    float ys[4], yc[4], bs[4], bc[4];
    bool inmap[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int pi = X0 + 8 * (q & 1) + li, pj = Y0 + 8 * (q >> 1) + lj;
        inmap[q] = (pi < Gm.npix) && (pj < Gm.npix);
        int64_t idx = (int64_t)pj * Gm.npix + pi;
        ys[q] = inmap[q] ? ymap[idx] : 0.0f;
        bs[q] = inmap[q] ? bmap[idx] : 0.0f;
        // the compensation carried over from earlier calls, when the caller keeps it
        yc[q] = (ycomp && inmap[q]) ? ycomp[idx] : 0.0f;
        bc[q] = (bcomp && inmap[q]) ? bcomp[idx] : 0.0f;
    }
    for (uint32_t p = p0; p < p1; ++p) {
        const uint32_t h = __builtin_amdgcn_readfirstlane(vals[p]);
        if (h >= (uint32_t)n) continue;
        const FlatRec &RF = rec[h];
        const FlatHead R = load_head(rec, h);
        const FootRec F = foot_uniform(R);
        const float *tab = tables + (int64_t)h * (kQ ? 2 * BP_MLP_NQ : BP_TAB_STRIDE);
        const int ox = X0 - R.cxi, oy = Y0 - R.cyi;   // tile corner relative to the centre pixel
        float sx[2], dys[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const float dx = (float)(ox + 8 * c + li) + R.hx;
            sx[c] = dx * dx;
            dys[c] = (float)(oy + 8 * c + lj) + R.hy;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int qx = q & 1, qy = q >> 1;
            const int pi = X0 + 8 * qx + li, pj = Y0 + 8 * qy + lj;
            const float dy = dys[qy];
            const float r2 = fmaf(dy, dy, sx[qx]);
            bool in = r2 < R.Rt2;
            // the FP32 distance is good to ~1e-6 relative: decide pixels that close to the edge
            // with the FP64 formula of the definition
            if (fabsf(r2 - R.Rt2) <= R.Rt2_band) in = inside_fp64(pi, pj, Gm.pix, RF.thx, RF.thy, RF.DA, RF.Rt);
            if (in && inmap[q]) {
                float u2 = R.ra2 - r2, U2 = R.rf2 - r2;
                // next to r_a (inside) or r_f the square root of a small difference needs the
                // difference in FP64; in zone B only the sign of u^2 is used
                if ((u2 > 0.0f && u2 < R.ra2_edge) || U2 < R.rf2_edge) {
                    double dxd = (double)(pi - R.cxi) + (0.5 - RF.cxd), dyd = (double)(pj - R.cyi) + (0.5 - RF.cyd);
                    double r2d = dxd * dxd + dyd * dyd;
                    u2 = (float)(RF.ra2d - r2d);
                    U2 = (float)(RF.rf2d - r2d);
                }
                float vp, vn;
                if (kQ) footprint_value_q(R, tab, r2, U2, &vp, &vn);
                else footprint_value(F, tab, r2, u2, U2, &vp, &vn);
                kahan_add(ys[q], yc[q], R.amp_y * vp);
                kahan_add(bs[q], bc[q], R.amp_b * vn);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (!inmap[q]) continue;
        const int pi = X0 + 8 * (q & 1) + li, pj = Y0 + 8 * (q >> 1) + lj;
        int64_t idx = (int64_t)pj * Gm.npix + pi;
        ymap[idx] = ys[q];
        bmap[idx] = bs[q];
        if (ycomp) ycomp[idx] = yc[q];
        if (bcomp) bcomp[idx] = bc[q];
    }
}

}  // namespace bp

using namespace bp;

template <bool kQ>
static int paste_flat_impl(const bp_params *p, int32_t npix, double pix_rad, int64_t n, const double *theta_x,
                                const double *theta_y, const double *v_los, const double *sol, const int32_t *status,
                                const float *tables, const float *meta, float *y_map, float *b_map, float *y_comp,
                                float *b_comp, void *ws, size_t ws_bytes, size_t *ws_needed, void *stream,
                                hipStream_t plan_stream = nullptr, hipEvent_t plan_done = nullptr) {
    if (check_params(p) || npix <= 0 || npix > 65536 || !(pix_rad > 0) || n < 0 || !ws_needed) return BP_E_ARG;
    if (n > 0 && (!theta_x || !theta_y || !v_los || !sol || !status || !tables || !meta)) return BP_E_ARG;
    if (!y_map || !b_map) return BP_E_ARG;
    if (n >= 0x7fffffffLL) return BP_E_OVERFLOW;
    hipStream_t s = (hipStream_t)stream;
    // set-up and plan run on plan_stream when one is given (its own dependencies set by the caller),
    // the deposit on stream after plan_done
    hipStream_t sp = plan_stream ? plan_stream : s;
    if (n == 0) { *ws_needed = 0; return BP_OK; }
    FlatGeom Gm;
    Gm.npix = npix;
    Gm.ntx = (npix + kTile - 1) / kTile;
    Gm.pix = pix_rad;
    const int64_t ntiles = (int64_t)Gm.ntx * Gm.ntx;
    // phase-1 layout
    Arena A1(nullptr, 0);
    A1.take<FlatRec>(n);
    A1.take<uint32_t>(n + 1);
    A1.take<uint32_t>(n + 1);
    A1.take<unsigned long long>(1);
    size_t phase1 = A1.used + scan_ws_bytes(n + 1);
    if (ws_bytes < phase1 || !ws) { *ws_needed = phase1 + 64; return BP_E_WORKSPACE; }
    Arena A(ws, ws_bytes);
    FlatRec *rec = A.take<FlatRec>(n);
    uint32_t *cnt = A.take<uint32_t>(n + 1);
    uint32_t *off = A.take<uint32_t>(n + 1);
    unsigned long long *total = A.take<unsigned long long>(1);
    void *scan_ws = (char *)ws + A.used;
    A.used += scan_ws_bytes(n + 1);
    // cleared with a fill kernel (a memset node misbehaves under graph replay on this target)
    if (fill_u32((uint32_t *)total, 0u, 2, sp)) return BP_E_HIP;
    if (fill_u32(cnt + n, 0u, 1, sp)) return BP_E_HIP;
    unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_flat_setup<kQ>, dim3(blocks), dim3(256), 0, sp, *p, Gm, n, theta_x, theta_y, v_los, sol, status,
                       meta, rec, cnt, total);
    if (hipGetLastError() != hipSuccess) return BP_E_HIP;
    unsigned long long np64 = 0;
    if (hipMemcpyAsync(&np64, total, sizeof(np64), hipMemcpyDeviceToHost, sp) != hipSuccess) return BP_E_HIP;
    if (hipStreamSynchronize(sp) != hipSuccess) return BP_E_HIP;
    if (np64 >= 0x7fffffffULL) return BP_E_OVERFLOW;
    const int64_t np = (int64_t)np64;
    // phase-2 layout (after the phase-1 part)
    size_t need = A.used;
    {
        Arena B(nullptr, 0);
        B.take<uint32_t>(np);
        B.take<uint32_t>(np);
        B.take<uint32_t>(np);
        B.take<uint32_t>(np);
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
    prof_begin(BP_PROF_FLAT_PLAN, sp);
    int e = scan_exclusive_u32(cnt, off, n + 1, scan_ws, sp);
    if (e) return e;
    hipLaunchKernelGGL(k_flat_emit, dim3(blocks), dim3(256), 0, sp, Gm, n, theta_x, theta_y, rec, off, k0, v0);
    if (hipGetLastError() != hipSuccess) return BP_E_HIP;
    int bits = 1;
    while ((1LL << bits) < ntiles) ++bits;
    bool in1 = false;
    e = radix_sort_u32(k0, v0, k1, v1, np, bits, sort_ws, sp, &in1);
    if (e) return e;
    uint32_t *ks = in1 ? k1 : k0, *vs = in1 ? v1 : v0;
    if (fill_u32(tst, 0u, ntiles, sp) || fill_u32(ten, 0u, ntiles, sp)) return BP_E_HIP;
    hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, sp, ks, np, tst, ten,
                       (uint32_t)ntiles);
    if (hipGetLastError() != hipSuccess) return BP_E_HIP;
    prof_end(BP_PROF_FLAT_PLAN, sp);
    if (sp != s) {
        if (hipEventRecord(plan_done, sp) != hipSuccess || hipStreamWaitEvent(s, plan_done, 0) != hipSuccess)
            return BP_E_HIP;
    }
    prof_begin(kQ ? BP_PROF_FLATQ_DEPOSIT : BP_PROF_FLAT_DEPOSIT, s);
    hipLaunchKernelGGL(k_flat_deposit<kQ>, dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, s, Gm, n, rec, tables, vs,
                       tst, ten, y_map, b_map, y_comp, b_comp, (int)ntiles);
    prof_end(kQ ? BP_PROF_FLATQ_DEPOSIT : BP_PROF_FLAT_DEPOSIT, s);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

extern "C" int bp_hp_paste_flat(const bp_params *p, int32_t npix, double pix_rad, int64_t n, const double *theta_x,
                                const double *theta_y, const double *v_los, const double *sol, const int32_t *status,
                                const float *tables, const float *meta, float *y_map, float *b_map, float *y_comp,
                                float *b_comp, void *ws, size_t ws_bytes, size_t *ws_needed, void *stream) {
    return paste_flat_impl<false>(p, npix, pix_rad, n, theta_x, theta_y, v_los, sol, status, tables, meta, y_map,
                                  b_map, y_comp, b_comp, ws, ws_bytes, ws_needed, stream);
}

extern "C" int bp_hp_paste_flat_q(const bp_params *p, int32_t npix, double pix_rad, int64_t n, const double *theta_x,
                                  const double *theta_y, const double *v_los, const double *sol, const int32_t *status,
                                  const float *qtables, const float *meta, float *y_map, float *b_map, float *y_comp,
                                  float *b_comp, void *ws, size_t ws_bytes, size_t *ws_needed, void *stream) {
    return paste_flat_impl<true>(p, npix, pix_rad, n, theta_x, theta_y, v_los, sol, status, qtables, meta, y_map,
                                 b_map, y_comp, b_comp, ws, ws_bytes, ws_needed, stream);
}

// ---------------------------------------------------------- one-call pipeline --
namespace {
constexpr int kMaxSideDevices = 64;
std::mutex g_side_mu;
SideStream g_side[kMaxSideDevices];
}  // namespace

int bp::side_stream_for_current_device(SideStream **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxSideDevices) return BP_E_HIP;
    std::lock_guard<std::mutex> lock(g_side_mu);
    SideStream &S = g_side[dev];
    if (!S.s) {
        // default priority: only the ordering changes, never the scheduling class
        hipStream_t st = nullptr;
        hipEvent_t e1 = nullptr, e2 = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return BP_E_HIP;
        if (hipEventCreateWithFlags(&e1, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&e2, hipEventDisableTiming) != hipSuccess) {
            if (e1) (void)hipEventDestroy(e1);
            (void)hipStreamDestroy(st);
            return BP_E_HIP;
        }
        S.meta_ready = e1;
        S.plan_done = e2;
        S.s = st;
    }
    *out = &S;
    return BP_OK;
}

int bp::join_side(SideStream *S, hipStream_t s, int e) {
    if (hipEventRecord(S->plan_done, S->s) != hipSuccess || hipStreamWaitEvent(s, S->plan_done, 0) != hipSuccess)
        return e ? e : BP_E_HIP;
    return e;
}

extern "C" int bp_hp_flat_pipeline(const bp_params *p, int32_t npix, double pix_rad, int64_t n, const double *M,
                                   const double *c, const double *z, const double *theta_x, const double *theta_y,
                                   const double *v_los, double *sol, int32_t *status, float *tables, float *meta,
                                   float *y_map, float *b_map, float *y_comp, float *b_comp, void *ws,
                                   size_t ws_bytes, size_t *ws_needed, void *stream) {
    if (check_params(p) || npix <= 0 || npix > 65536 || !(pix_rad > 0) || n < 0 || !ws_needed) return BP_E_ARG;
    if (!y_map || !b_map) return BP_E_ARG;
    if (n > 0 && (!M || !c || !z || !theta_x || !theta_y || !v_los || !sol || !status || !tables || !meta))
        return BP_E_ARG;
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
    e = paste_flat_impl<false>(p, npix, pix_rad, n, theta_x, theta_y, v_los, sol, status, tables, meta, y_map, b_map,
                               y_comp, b_comp, ws, ws_bytes, ws_needed, stream, S->s, S->plan_done);
    return e ? join_side(S, s, e) : BP_OK;
}

int bp::paste_flat_q_planned(const bp_params *p, int32_t npix, double pix_rad, int64_t n, const double *theta_x,
                             const double *theta_y, const double *v_los, const double *sol, const int32_t *status,
                             const float *qtables, const float *meta, float *y_map, float *b_map, float *y_comp,
                             float *b_comp, void *ws, size_t ws_bytes, size_t *ws_needed, hipStream_t stream,
                             hipStream_t plan_stream, hipEvent_t plan_done) {
    return paste_flat_impl<true>(p, npix, pix_rad, n, theta_x, theta_y, v_los, sol, status, qtables, meta, y_map,
                                 b_map, y_comp, b_comp, ws, ws_bytes, ws_needed, stream, plan_stream, plan_done);
}

// ------------------------------------------------------ allocation-free variant --
// The workspace of bp_hp_paste_flat_noalloc: a fixed device array, one copy per GPU for the life of the
// process.  Host code never uses this symbol as an address (it names a host-side stand-in): the device
// address comes from hipGetSymbolAddress, once per device, and is what the kernels receive.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on the current device (looked up on its first use there)
int scratch_for_current_device(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BP_E_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return BP_E_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return BP_OK;
}
}  // namespace

extern "C" size_t bp_hp_paste_flat_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" int bp_hp_paste_flat_noalloc(const bp_params *p, int32_t npix, double pix_rad, int64_t n,
                                        const double *theta_x, const double *theta_y, const double *v_los,
                                        const double *sol, const int32_t *status, const float *tables,
                                        const float *meta, float *y_map, float *b_map, float *y_comp, float *b_comp,
                                        size_t *scratch_needed, void *stream) {
    void *ptr = nullptr;
    int e = scratch_for_current_device(&ptr);
    if (e) return e;
    size_t need = 0;
    e = paste_flat_impl<false>(p, npix, pix_rad, n, theta_x, theta_y, v_los, sol, status, tables, meta, y_map, b_map,
                               y_comp, b_comp, ptr, kScratchBytes, &need, stream);
    if (scratch_needed) *scratch_needed = need;
    return e;
}
