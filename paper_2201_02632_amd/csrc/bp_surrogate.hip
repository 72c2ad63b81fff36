// Surrogate data path: network features, training targets from the exact
// solve, column statistics, batch gathering, the loss gradient, and the
// inference epilogue that turns network outputs into deposit tables.
#include <hip/hip_runtime.h>
#include <math.h>

#include "bp_device.hpp"
#include "bp_footprint.hpp"
#include "bp_internal.hpp"

namespace bp {

// normalised inputs: log10 M in [12.5, 15.5], ln c in [ln 2, ln 15], z in [0.05, 3] -> about [-1, 1]
__global__ void k_features(int64_t n, const double *__restrict__ M, const double *__restrict__ c,
                           const double *__restrict__ z, float *__restrict__ x) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double lc0 = 0.5 * (log(2.0) + log(15.0)), lch = 0.5 * (log(15.0) - log(2.0));
    float *r = x + i * BP_MLP_IN;
    r[0] = (float)((log10(M[i]) - 14.0) / 1.5);
    r[1] = (float)((log(c[i]) - lc0) / lch);
    r[2] = (float)((z[i] - 1.525) / 1.475);
    for (int k = 3; k < BP_MLP_IN; ++k) r[k] = 0.0f;
}

__host__ __device__ inline double qnode(int k) { return 0.5 * (1.0 - cos(kPi * k / (BP_MLP_NQ - 1))); }

// record in units of R_t for evaluating the exact zone tables at q = r_perp / R_t
struct UnitRec {
    float Rt2, ra, ra2, rv2, rf, rf2, D, isqD, r2min;
    float eta_lo, eta_ih, om_lo, om_ih, ze_lo, ze_ih;
    int32_t flags;
};

// electron-density scale [1/cm^3]: the cosmic baryon share of the mean density inside r_vir, as
// fully ionised electrons.  The network predicts n_e0 relative to it (and P_e0 relative to the
// surface pressure), which keeps the amplitude targets within a narrow range.
__device__ inline double ne_scale(const bp_params &P, double M, double rv) {
    const double u_len = kMpc / P.h, u_mass = kMsun / P.h;
    const double r = rv * u_len;
    const double rho = M * u_mass / (4.0 * kPi / 3.0 * r * r * r);
    return (P.Omega_b / P.Omega_m) * rho / (2.0 / (1.0 + P.X_H) * kMp);
}

// one thread per (halo, q node); thread k = 0 also writes the scalars and padding
__global__ void k_targets(bp_params P, int64_t n, const double *__restrict__ sol, const int32_t *__restrict__ status,
                          const float *__restrict__ tables, const float *__restrict__ meta, float *__restrict__ t) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * BP_MLP_NQ) return;
    int64_t i = e / BP_MLP_NQ;
    int k = (int)(e % BP_MLP_NQ);
    float *row = t + i * BP_MLP_OUT;
    auto S = [&](int f) { return sol[(int64_t)f * n + i]; };
    auto Mt = [&](int f) { return meta[(int64_t)f * n + i]; };
    if (status[i] & ~BP_S_MULTI_ROOT) {
        const float nanv = __int_as_float(0x7fc00000);
        row[k] = nanv; row[BP_MLP_NQ + k] = nanv;
        if (k == 0)
            for (int q = 2 * BP_MLP_NQ; q < BP_MLP_OUT; ++q) row[q] = q < BP_MLP_NOUT ? nanv : 0.0f;
        return;
    }
    const double Rt = S(BP_SOL_RT), rv = S(BP_SOL_RVIR) / Rt, rf = S(BP_SOL_RF) / Rt, ra = fmin(rv, rf);
    UnitRec R;
    R.Rt2 = 1.0f;
    R.ra = (float)ra; R.ra2 = (float)(ra * ra); R.rv2 = (float)(rv * rv);
    R.rf = (float)rf; R.rf2 = (float)(rf * rf);
    const bool shell = rf > rv;
    const double D = shell ? rf * rf - rv * rv : 0.0;
    R.D = (float)D; R.isqD = D > 0.0 ? (float)(1.0 / sqrt(D)) : 0.0f;
    R.r2min = (float)(1e-10 * ra * ra);
    float elo = Mt(BP_META_ETA_LO), ehi = Mt(BP_META_ETA_HI), olo = Mt(BP_META_OM_LO), ohi = Mt(BP_META_OM_HI),
          zlo = Mt(BP_META_ZE_LO), zhi = Mt(BP_META_ZE_HI);
    set_zone_grids(R, elo, ehi, olo, ohi, zlo, zhi);
    R.flags = (shell ? 1 : 0) | ((1.0 > rv) ? 2 : 0) | 4;
    double q = qnode(k);
    if (k == BP_MLP_NQ - 1) q = 1.0 - 1e-6;   // the edge node: the limit from inside
    double r2 = q * q;
    float vp, vn;
    footprint_value(R, tables + i * BP_TAB_STRIDE, (float)r2, (float)(ra * ra - r2), (float)(rf * rf - r2), &vp, &vn);
    double E = sqrt(fmax(1.0 - r2 / (rf * rf), 0.0));
    row[k] = (float)log((double)vp / E);
    row[BP_MLP_NQ + k] = (float)log((double)vn / E);
    if (k == 0) {
        row[2 * BP_MLP_NQ + 0] = (float)log(S(BP_SOL_XF));
        row[2 * BP_MLP_NQ + 1] = (float)log((double)Mt(BP_META_PE0) / S(BP_SOL_PS));
        row[2 * BP_MLP_NQ + 2] = (float)log((double)Mt(BP_META_NE0) / ne_scale(P, S(BP_SOL_M), S(BP_SOL_RVIR)));
        for (int q2 = BP_MLP_NOUT; q2 < BP_MLP_OUT; ++q2) row[q2] = 0.0f;
    }
}

// column mean and standard deviation over rows with finite values (FP64 sums, fixed order)
// One workgroup per column: lane l sums rows l, l + 256, ... in order, then a fixed tree over the
// lanes (FP64 sums; non-finite targets are skipped).
__global__ void __launch_bounds__(256) k_stats(int64_t n, const float *__restrict__ t, float *__restrict__ mean,
                                               float *__restrict__ sd) {
    __shared__ double rs[256], rs2[256];
    __shared__ int64_t rc[256];
    const int c = blockIdx.x;
    double s = 0.0, s2 = 0.0;
    int64_t cnt = 0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        float v = t[i * BP_MLP_OUT + c];
        if (!isfinite(v)) continue;
        s += v; s2 += (double)v * v; ++cnt;
    }
    rs[threadIdx.x] = s; rs2[threadIdx.x] = s2; rc[threadIdx.x] = cnt;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            rs[threadIdx.x] += rs[threadIdx.x + w];
            rs2[threadIdx.x] += rs2[threadIdx.x + w];
            rc[threadIdx.x] += rc[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t m = rc[0];
        const double mu = m ? rs[0] / m : 0.0;
        const double var = m ? rs2[0] / m - mu * mu : 0.0;
        mean[c] = (float)mu;
        sd[c] = (c < BP_MLP_NOUT && var > 1e-20) ? (float)sqrt(var) : 1.0f;
    }
}

__global__ void k_gather(int64_t n, int cols, const float *__restrict__ in, const int64_t *__restrict__ idx,
                         float *__restrict__ out) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * cols) return;
    int64_t i = e / cols;
    int c = (int)(e % cols);
    out[e] = in[idx[i] * cols + c];
}

// counter-based batch sampling (SplitMix64 of seed, step, row): row i of the batch is data row
// (hash >> 11) mod n_data
// loss gradient for the standardised targets, one wave per row (lanes stride the columns);
// rows with a non-finite target contribute nothing
__global__ void k_mse(int64_t n, const float *__restrict__ y, const float *__restrict__ t,
                      const float *__restrict__ mean, const float *__restrict__ sd, float *__restrict__ dy,
                      float *__restrict__ loss) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (i >= n) return;   // whole wave leaves together
    constexpr int kPer = (BP_MLP_OUT + 63) / 64;
    // weights: 1 per table entry, kAuxWeight for each of x_f, P_e0, n_e0 (they scale the whole footprint)
    const float kAuxWeight = 16.0f;
    const float wsum = 2.0f * BP_MLP_NQ + 3.0f * kAuxWeight;
    const float scale = 2.0f / ((float)n * wsum);
    float tv[kPer];
    bool fin = true;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        int c = lane + 64 * j;
        tv[j] = c < BP_MLP_NOUT ? t[i * BP_MLP_OUT + c] : 0.0f;
        fin = fin && isfinite(tv[j]);
    }
    const bool ok = __all(fin);
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        int c = lane + 64 * j;
        if (c >= BP_MLP_OUT) break;
        float d = 0.0f;
        if (ok && c < BP_MLP_NOUT) {
            float wc = (c >= 2 * BP_MLP_NQ) ? kAuxWeight : 1.0f;
            float r = y[i * BP_MLP_OUT + c] - (tv[j] - mean[c]) / sd[c];
            acc += wc * r * r;
            d = scale * wc * r;
        }
        dy[i * BP_MLP_OUT + c] = d;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) loss[i] = acc;
}

// The loss of one training step, fused: rows drawn by train_row (targets gathered here), the loss
// gradient written straight as the BF16 operand of the backward, and the b4 gradient left as
// per-64-row column partials b4p[chunk][c] (wavefront w of the chunk's eight takes rows w, w + 8, ..,
// in order, and the wavefronts are combined in order).  Same weights and formula as k_mse.  One
// workgroup of 512 threads per 64-row chunk.
constexpr int kMseWaves = 8, kMseRows = 64 / kMseWaves;
__global__ void __launch_bounds__(512) k_mse_train(int64_t n, int64_t ndata, uint64_t seed, int64_t step,
                                                   const float *__restrict__ y, const float *__restrict__ tdata,
                                                   const float *__restrict__ mean, const float *__restrict__ sd,
                                                   uint16_t *__restrict__ g4, float *__restrict__ b4p,
                                                   float *__restrict__ loss) {
    __shared__ float red[kMseWaves][BP_MLP_OUT];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    constexpr int kPer = (BP_MLP_OUT + 63) / 64;
    const float kAuxWeight = 16.0f;
    const float wsum = 2.0f * BP_MLP_NQ + 3.0f * kAuxWeight;
    const float scale = 2.0f / ((float)n * wsum);
    float mc[kPer], sdc[kPer], wc[kPer], col[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int c = lane + 64 * j;
        const bool used = c < BP_MLP_NOUT;
        mc[j] = used ? mean[c] : 0.0f;
        sdc[j] = used ? sd[c] : 1.0f;
        wc[j] = (c >= 2 * BP_MLP_NQ) ? kAuxWeight : 1.0f;
        col[j] = 0.0f;
    }
    const int64_t r0 = (int64_t)blockIdx.x * 64 + w;   // this wavefront's rows: r0 + kMseWaves q
    // lane q < kMseRows draws the data row of row q (one 64-bit modulo per lane), read back by shuffles
    const int64_t mine = r0 + kMseWaves * (int64_t)lane;
    const int64_t src_l = (lane < kMseRows && mine < n) ? train_row(seed, step, mine, ndata) : 0;
    float tv[kMseRows][kPer], yv[kMseRows][kPer];
#pragma unroll
    for (int q = 0; q < kMseRows; ++q) {
        const int64_t i = r0 + kMseWaves * q;
        const int64_t src = (int64_t)(((uint64_t)(uint32_t)__shfl((int)(src_l >> 32), q, 64) << 32) |
                                      (uint32_t)__shfl((int)src_l, q, 64));
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int c = lane + 64 * j;
            const bool ld = i < n && c < BP_MLP_NOUT;
            tv[q][j] = ld ? tdata[src * BP_MLP_OUT + c] : 0.0f;
            yv[q][j] = ld ? y[i * BP_MLP_OUT + c] : 0.0f;
        }
    }
#pragma unroll
    for (int q = 0; q < kMseRows; ++q) {
        const int64_t i = r0 + kMseWaves * q;
        if (i >= n) break;   // wave-uniform
        bool fin = true;
#pragma unroll
        for (int j = 0; j < kPer; ++j) fin = fin && isfinite(tv[q][j]);
        const bool ok = __all(fin);
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int c = lane + 64 * j;
            if (c >= BP_MLP_OUT) break;
            float d = 0.0f;
            if (ok && c < BP_MLP_NOUT) {
                const float r = yv[q][j] - (tv[q][j] - mc[j]) / sdc[j];
                acc += wc[j] * r * r;
                d = scale * wc[j] * r;
            }
            g4[i * BP_MLP_OUT + c] = f2bf(d);
            col[j] += d;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) loss[i] = acc;
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int c = lane + 64 * j;
        if (c < BP_MLP_OUT) red[w][c] = col[j];
    }
    __syncthreads();
    for (int c = threadIdx.x; c < BP_MLP_OUT; c += blockDim.x) {
        float t = red[0][c];
#pragma unroll
        for (int v = 1; v < kMseWaves; ++v) t += red[v][c];
        b4p[(int64_t)blockIdx.x * BP_MLP_OUT + c] = t;
    }
}

// network output -> q-tables (G values): one thread per (halo, 4 q nodes), 16-byte loads and
// stores (rows of BP_MLP_OUT and 2 BP_MLP_NQ floats keep every group of four aligned)
static_assert(BP_MLP_OUT % 4 == 0 && (2 * BP_MLP_NQ) % 4 == 0, "16-byte groups");
__global__ void k_apply_q(int64_t n, const float *__restrict__ y, const float *__restrict__ mean,
                          const float *__restrict__ sd, const int32_t *__restrict__ status,
                          const uint32_t *__restrict__ skip, float *__restrict__ qt) {
    constexpr int G4 = 2 * BP_MLP_NQ / 4;
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * G4) return;
    int64_t i = e / G4;
    int k = 4 * (int)(e % G4);
    // a halo marked in skip is left alone, its status not even read (another stream may be writing it)
    if ((skip && skip[i]) || status[i]) return;
    const float4 r = *reinterpret_cast<const float4 *>(y + i * BP_MLP_OUT + k);
    const float4 s = *reinterpret_cast<const float4 *>(sd + k);
    const float4 m = *reinterpret_cast<const float4 *>(mean + k);
    float4 g;
    g.x = __expf(r.x * s.x + m.x);
    g.y = __expf(r.y * s.y + m.y);
    g.z = __expf(r.z * s.z + m.z);
    g.w = __expf(r.w * s.w + m.w);
    *reinterpret_cast<float4 *>(qt + i * 2 * BP_MLP_NQ + k) = g;
}

// meta (PE0, NE0) of a halo solved by the seeded solve: the central electron pressure and density of
// Sec. 3.2 from the solved P0 and rho0, as the exact tables' set-up writes them.  One thread per halo:
// a launch of its own, so that this FP64 work does not run on one lane of a wavefront while the
// other 63 wait.
__global__ void k_apply_halo(bp_params P, int64_t n, const double *__restrict__ sol, const int32_t *__restrict__ status,
                             float *__restrict__ meta) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || status[i]) return;
    const double X = P.X_H;
    meta[(int64_t)BP_META_PE0 * n + i] = (float)((2.0 * X + 2.0) / (5.0 * X + 3.0) * sol[(int64_t)BP_SOL_P0 * n + i]);
    meta[(int64_t)BP_META_NE0 * n + i] = (float)(sol[(int64_t)BP_SOL_RHO0 * n + i] / (2.0 / (1.0 + X) * kMp));
    for (int f = 0; f < BP_META_PE0; ++f) meta[(int64_t)f * n + i] = 0.0f;
    for (int f = BP_META_PR_RV; f < BP_META_NFIELDS; ++f) meta[(int64_t)f * n + i] = 0.0f;
}

}  // namespace bp

using namespace bp;

static inline unsigned nblk(int64_t work) { return (unsigned)((work + 255) / 256); }

extern "C" int bp_surrogate_features(int64_t n, const double *M, const double *c, const double *z, float *x,
                                     void *stream) {
    if (n < 0 || (n > 0 && (!M || !c || !z || !x))) return BP_E_ARG;
    if (n == 0) return BP_OK;
    hipLaunchKernelGGL(k_features, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, n, M, c, z, x);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

extern "C" int bp_surrogate_targets(const bp_params *p, int64_t n, const double *sol, const int32_t *status,
                                    const float *tables, const float *meta, float *targets, void *stream) {
    if (check_params(p) || n < 0 || (n > 0 && (!sol || !status || !tables || !meta || !targets))) return BP_E_ARG;
    if (n == 0) return BP_OK;
    hipLaunchKernelGGL(k_targets, dim3(nblk(n * BP_MLP_NQ)), dim3(256), 0, (hipStream_t)stream, *p, n, sol, status,
                       tables, meta, targets);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

extern "C" int bp_surrogate_stats(int64_t n, const float *targets, float *mean, float *std, void *stream) {
    if (n <= 0 || !targets || !mean || !std) return BP_E_ARG;
    hipLaunchKernelGGL(k_stats, dim3(BP_MLP_OUT), dim3(256), 0, (hipStream_t)stream, n, targets, mean, std);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

extern "C" int bp_gather_rows(int64_t n, int32_t cols, const float *in, const int64_t *idx, float *out, void *stream) {
    if (n < 0 || cols <= 0 || (n > 0 && (!in || !idx || !out))) return BP_E_ARG;
    if (n == 0) return BP_OK;
    hipLaunchKernelGGL(k_gather, dim3(nblk(n * cols)), dim3(256), 0, (hipStream_t)stream, n, cols, in, idx, out);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

extern "C" int bp_surrogate_mse(int64_t n, const float *y, const float *targets, const float *mean, const float *std,
                                float *dy, float *loss_rows, void *stream) {
    if (n <= 0 || !y || !targets || !mean || !std || !dy || !loss_rows) return BP_E_ARG;
    hipLaunchKernelGGL(k_mse, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, (hipStream_t)stream, n, y, targets, mean, std, dy,
                       loss_rows);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

int bp::surrogate_apply_q(int64_t n, const float *y, const float *mean, const float *std, const int32_t *status,
                          const uint32_t *skip, float *qtables, hipStream_t s) {
    if (n == 0) return BP_OK;
    prof_begin(BP_PROF_SURR_APPLY, s);
    hipLaunchKernelGGL(k_apply_q, dim3(nblk(n * 2 * BP_MLP_NQ / 4)), dim3(256), 0, s, n, y, mean, std, status, skip,
                       qtables);
    prof_end(BP_PROF_SURR_APPLY, s);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

int bp::surrogate_apply_meta(const bp_params *p, int64_t n, const double *sol, const int32_t *status, float *meta,
                             hipStream_t s) {
    if (n == 0) return BP_OK;
    prof_begin(BP_PROF_SURR_APPLY, s);
    hipLaunchKernelGGL(k_apply_halo, dim3(nblk(n)), dim3(256), 0, s, *p, n, sol, status, meta);
    prof_end(BP_PROF_SURR_APPLY, s);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

extern "C" int bp_surrogate_apply(const bp_params *p, int64_t n, const float *y, const float *mean, const float *std,
                                  const double *sol, const int32_t *status, float *qtables, float *meta, void *stream) {
    if (check_params(p) || n < 0 || (n > 0 && (!y || !mean || !std || !sol || !status || !qtables || !meta)))
        return BP_E_ARG;
    if (n == 0) return BP_OK;
    if (((uintptr_t)y | (uintptr_t)mean | (uintptr_t)std | (uintptr_t)qtables) & 15) return BP_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    int e = surrogate_apply_q(n, y, mean, std, status, nullptr, qtables, s);
    return e ? e : surrogate_apply_meta(p, n, sol, status, meta, s);
}

extern "C" size_t bp_surrogate_train_ws_bytes(int64_t batch) {
    if (batch <= 0) return 0;
    return (size_t)batch * (BP_MLP_IN + BP_MLP_OUT + 1) * 4 + bp_mlp_act_bytes(batch) +
           bp_mlp_backward_ws_bytes(batch) + 8 * 256;
}

// One step: forward of the drawn batch (layer 1 gathers its rows), the fused loss, the backward in
// three launches, and Adam from the gradient's partials: nine launches.
extern "C" int bp_surrogate_train(float *w, uint16_t *w_bf16, float *m, float *v, float *grad, const float *mean,
                                  const float *std, int64_t ndata, const float *x, const float *targets, int64_t steps,
                                  int64_t batch, float lr0, float lr1, uint64_t seed, int64_t step0, float *loss_rows,
                                  void *ws, size_t ws_bytes, void *stream) {
    if (!w || !w_bf16 || !m || !v || !grad || !mean || !std || !x || !targets || !ws || ndata <= 0 || steps < 0 ||
        batch <= 0 || step0 < 0)
        return BP_E_ARG;
    if (ws_bytes < bp_surrogate_train_ws_bytes(batch)) return BP_E_WORKSPACE;
    if (((uintptr_t)ws % 256) || ((uintptr_t)x % 16)) return BP_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    Arena A(ws, ws_bytes);
    float *xb = A.take<float>(batch * BP_MLP_IN), *y = A.take<float>(batch * BP_MLP_OUT);
    float *loss = loss_rows ? loss_rows : A.take<float>(batch);
    void *act = A.take<char>(bp_mlp_act_bytes(batch));
    const size_t bwb = bp_mlp_backward_ws_bytes(batch);
    void *bws = A.take<char>(bwb);
    uint16_t *g4 = nullptr;
    GradParts parts;
    int e = mlp_backward_layout(bws, bwb, batch, &g4, &parts);
    if (e) return e;
    const unsigned chunks = (unsigned)((batch + 63) / 64);
    for (int64_t k = 0; k < steps; ++k) {
        e = mlp_forward_train(w, w_bf16, batch, ndata, seed, step0 + k, x, xb, act, y, s);
        if (e) return e;
        hipLaunchKernelGGL(k_mse_train, dim3(chunks), dim3(64 * kMseWaves), 0, s, batch, ndata, seed, step0 + k, y, targets, mean,
                           std, g4, (float *)parts.b4, loss);
        e = mlp_backward_g4(w_bf16, batch, xb, act, bws, bwb, s);
        if (e) return e;
        double frac = steps > 1 ? (double)k / (double)(steps - 1) : 1.0;
        float lr = (float)(lr1 + 0.5 * (lr0 - lr1) * (1.0 + cos(kPi * frac)));
        e = mlp_adam_parts(parts, w, m, v, grad, w_bf16, lr, 0.9f, 0.999f, 1e-8f, step0 + k + 1, s);
        if (e) return e;
    }
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}
