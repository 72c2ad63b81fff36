// K10-K12: the profile-table surrogate network, forward, backward and Adam.
//
// Network (inputs normalised (log10 M, ln c, z)):
//   z1 = W1 x + b1                       FP32 (3 inputs: VALU)
//   h1 = bf16(silu(z1))
//   z2 = W2 h1 + b2, h2 = bf16(silu(z2)) BF16 MFMA, FP32 accumulation
//   z3 = W3 h2 + b3, h3 = bf16(silu(z3))
//   y  = W4 h3 + b4                      FP32 output
// The hidden-layer products run on gfx950's v_mfma_f32_16x16x32_bf16 (a 16x16
// block over 32 k per instruction): a workgroup computes a 64x64 output tile
// with four wavefronts (2x2 blocks of 16x16 each), staging the tile's whole K
// range in LDS at once.  Weight gradients reduce over the batch with split-K
// partial tiles, bias gradients with per-64-row column partials, all summed in
// a fixed order, so training is deterministic.
#include <hip/hip_runtime.h>
#include <math.h>

#include "bp_device.hpp"
#include "bp_internal.hpp"

namespace bp {

typedef short sx4 __attribute__((ext_vector_type(4)));
typedef float fx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// D (16x16, FP32) += A (16x32) B (32x16) in BF16.  Lane l supplies A[l % 16][8 (l / 16) .. + 7] and
// B[8 (l / 16) .. + 7][l % 16] (eight consecutive k each) and holds D[4 (l / 16) + j][l % 16], j < 4.
__device__ inline fx4 mfma32(const bf16x8 &a, const bf16x8 &b, const fx4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ inline sx4 pack_bf4(float a, float b, float c, float d) {
    sx4 r;
    r[0] = (short)f2bf(a); r[1] = (short)f2bf(b); r[2] = (short)f2bf(c); r[3] = (short)f2bf(d);
    return r;
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// SiLU and its derivative with the hardware exponential and reciprocal (about 1 ulp each)
__device__ inline float sigmoid(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ inline float silu(float z) { return z * sigmoid(z); }
__device__ inline float dsilu(float z) {
    float s = sigmoid(z);
    return s * (1.0f + z * (1.0f - s));
}

enum { EPI_BIAS_SILU = 0, EPI_BIAS = 1, EPI_DSILU = 2, EPI_PARTIAL = 3 };

struct GemmArgs {
    int64_t M, N, K;
    const uint16_t *A; int64_t a_m, a_k;   // A(m,k) = A[m*a_m + k*a_k]
    const uint16_t *B; int64_t b_k, b_n;   // B(k,n) = B[k*b_k + n*b_n]
    const float *bias;                      // EPI_BIAS*: [N]
    float *Z; int64_t ldz;                  // EPI_BIAS_SILU: pre-activation out (optional); EPI_DSILU: in
    uint16_t *H; int64_t ldh;               // bf16 output (EPI_BIAS_SILU, EPI_DSILU)
    float *F; int64_t ldf;                  // fp32 output (EPI_BIAS: y; EPI_DSILU: g*silu'(z) optional; PARTIAL)
    int64_t kchunk;                         // split-K chunk (PARTIAL), else K
    float *cs;                              // EPI_DSILU: per-64-row column sums of the output (optional)
    const float *xs;                        // EPI_DSILU with cs: also sums weighted by inputs x[m][0..2]
    int64_t ks;                             // split-K slices (the grid's third tile dimension)
    // Layer 1 fused into the A staging of layer 2 (A = h1 computed from x, K = 256):
    const float *x1;                        // inputs [.][BP_MLP_IN]: row m, or row train_row(m) if ndata > 0
    const float *W1, *b1;
    float *Z1; uint16_t *H1;                // z1 and h1 [M][256], stored by the tiles of the first column block
    float *xb;                              // with ndata > 0: the drawn rows' first BP_MLP_NIN inputs, [M][BP_MLP_IN]
    int64_t ndata, step; uint64_t seed;
};

// 64x64 output tile per workgroup; the four wavefronts cover it 2x2, 32x32 each (2x2 blocks of 16x16).
// A tile's K range is staged in LDS kGKC = 256 k at a time, all loads of a stage issued together, so
// a tile waits on memory once per 256 k rather than once per MFMA step (the K of every product here
// is 144 or 256, or a split-K slice of the batch of at most 256).  Both operands sit in LDS with k
// contiguous; an operand contiguous in m (or n) is transposed 8x8 in registers on its way in.  The
// MFMA takes the B tile as its first operand, so a lane's accumulator holds four consecutive output
// columns of one row and the epilogue moves them as one vector.  Every operand dimension that is
// loaded 16 bytes at a time is a multiple of 8 (checked at launch); k beyond K and rows beyond M are
// zero-filled.
constexpr int kGM = 64, kGN = 64, kGKC = 256, kGLd = kGKC;   // LDS row: 256 bf16 = 32 groups of 16 bytes
constexpr int kBK = 32;                                       // k per MFMA step

typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// The 16-byte group g of LDS row r is stored at group g ^ swz(r).  LDS serves a 16-byte access 16
// lanes at a time over 64 four-byte banks, so the 16 lanes must touch 16 different groups mod 16; with
// this swizzle they do for every pattern used here: 16 consecutive rows at one group (the MFMA
// fragments), one row at 16 consecutive groups (row-major staging), and the rows 8a + j (a < 8) at
// two neighbouring groups (transposed staging).
__device__ inline int swz(int r) { return (r ^ (r >> 3)) & 15; }
__device__ inline uint16_t *lds_at(uint16_t (*s)[kGLd], int r, int k) { return &s[r][((k >> 3) ^ swz(r)) << 3]; }

// Rows r0 .. r0+63 of an operand contiguous in k (element (r, k) at src[r * ld + k]), k in
// [k0, k0 + 256) clipped to kend, into row r, column k - k0 of dst (swizzled, lds_at).
__device__ inline void stage_kmajor(const uint16_t *__restrict__ src, int64_t ld, int64_t r0, int64_t rend,
                                    int64_t k0, int64_t kend, uint16_t (*dst)[kGLd], int t) {
    u16x8 v[8];
    const u16x8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int e = t + 256 * i, r = e >> 5, kq = (e & 31) * 8;
        const int64_t gr = r0 + r, gk = k0 + kq;
        v[i] = (gr < rend && gk < kend) ? *(const u16x8 *)(src + gr * ld + gk) : zero8;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int e = t + 256 * i, r = e >> 5, kq = (e & 31) * 8;
        *(u16x8 *)lds_at(dst, r, kq) = v[i];
    }
}

// The same for an operand contiguous in r (element (r, k) at src[k * ld + r]): thread t reads the
// 8x8 block of rows 8 (t % 8) .. + 7 and k 8 (t / 8) .. + 7 and writes it transposed.
__device__ inline void stage_rmajor(const uint16_t *__restrict__ src, int64_t ld, int64_t r0, int64_t rend,
                                    int64_t k0, int64_t kend, uint16_t (*dst)[kGLd], int t) {
    const int rq = (t & 7) * 8, kq = (t >> 3) * 8;
    const int64_t gr = r0 + rq;
    u16x8 v[8];
    const u16x8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int64_t gk = k0 + kq + i;
        v[i] = (gr < rend && gk < kend) ? *(const u16x8 *)(src + gk * ld + gr) : zero8;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        u16x8 o;
#pragma unroll
        for (int i = 0; i < 8; ++i) o[i] = v[i][j];
        *(u16x8 *)lds_at(dst, rq + j, kq) = o;
    }
}

__device__ inline void st_bf4(uint16_t *p, float a, float b, float c, float d) { *(sx4 *)p = pack_bf4(a, b, c, d); }

// first layer in FP32: z1 = b1 + sum_q W1[.][q] x[q] (in q order), h1 = bf16(silu(z1))
__device__ inline float layer1_z(float b, const float (&wq)[BP_MLP_NIN], const float (&x)[BP_MLP_NIN]) {
    float v = b;
#pragma unroll
    for (int q = 0; q < BP_MLP_NIN; ++q) v += wq[q] * x[q];
    return v;
}

// The A tile of layer 2 (rows r0 .. r0+63, all 256 k) computed from the inputs instead of loaded:
// thread t always makes the eight outputs k = 8 (t % 32) .. + 7, for rows t / 32 + 8 i.  With
// store set, z1 and h1 (and the drawn rows' first BP_MLP_NIN inputs) also go to memory for the
// backward.  All input loads are issued before the first store.
__device__ inline void stage_layer1(const GemmArgs &g, int64_t r0, bool store, uint16_t (*dst)[kGLd], int t) {
    const int kq = (t & 31) * 8, lane = t & 63;
    float bv[8], wv[8][BP_MLP_NIN];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        bv[j] = g.b1[kq + j];
#pragma unroll
        for (int q = 0; q < BP_MLP_NIN; ++q) wv[j][q] = g.W1[(kq + j) * BP_MLP_IN + q];
    }
    // the wavefront's rows are t / 32 + 8 i for its two values of t / 32: lane l < 16 draws the data
    // row of row (2 (t / 64) + l % 2) + 8 (l / 2), read back by shuffles
    int64_t src_l = 0;
    if (g.ndata > 0 && lane < 16) {
        const int64_t m = r0 + 2 * (t >> 6) + (lane & 1) + 8 * (lane >> 1);
        if (m < g.M) src_l = train_row(g.seed, g.step, m, g.ndata);
    }
    float xr[8][BP_MLP_NIN];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int64_t m = r0 + (t >> 5) + 8 * i;
        int64_t src = m;
        if (g.ndata > 0) {
            const int from = ((t >> 5) & 1) + 2 * i;
            src = (int64_t)(((uint64_t)(uint32_t)__shfl((int)(src_l >> 32), from, 64) << 32) |
                            (uint32_t)__shfl((int)src_l, from, 64));
        }
#pragma unroll
        for (int q = 0; q < BP_MLP_NIN; ++q) xr[i][q] = m < g.M ? g.x1[src * BP_MLP_IN + q] : 0.0f;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int r = (t >> 5) + 8 * i;
        const int64_t m = r0 + r;
        u16x8 h = {0, 0, 0, 0, 0, 0, 0, 0};
        if (m < g.M) {
            fx4 z0, z1;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                z0[j] = layer1_z(bv[j], wv[j], xr[i]);
                z1[j] = layer1_z(bv[4 + j], wv[4 + j], xr[i]);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                h[j] = f2bf(silu(z0[j]));
                h[4 + j] = f2bf(silu(z1[j]));
            }
            if (store) {
                *(fx4 *)(g.Z1 + m * BP_MLP_HID + kq) = z0;
                *(fx4 *)(g.Z1 + m * BP_MLP_HID + kq + 4) = z1;
                *(u16x8 *)(g.H1 + m * BP_MLP_HID + kq) = h;
                if (g.xb && kq == 0)
#pragma unroll
                    for (int q = 0; q < BP_MLP_NIN; ++q) g.xb[m * BP_MLP_IN + q] = xr[i][q];
            }
        }
        *(u16x8 *)lds_at(dst, r, kq) = h;
    }
}

// One 64x64 tile (linear index id over M tiles, then N tiles, then split-K slices).
// kAK: A contiguous in k (a_k == 1), else in m (a_m == 1); kBK1: B contiguous in k (b_k == 1), else in n.
// Workgroups are dealt to the eight XCDs round-robin by id.  With ks a multiple of 8 the split-K
// slices are dealt out whole: all tiles of slice bz run on XCD bz % 8, so each slice's operand rows
// are fetched into one L2 only.  Otherwise the tiles of one row block (all column blocks) share an XCD
// whenever the number of row blocks is a multiple of 8.
template <int EPI, bool kAK, bool kBK1, bool kL1 = false>
__device__ inline void gemm_tile(const GemmArgs &g, int64_t id, uint16_t (*As)[kGLd], uint16_t (*Bs)[kGLd]) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
    const int64_t mt = (g.M + kGM - 1) / kGM, nt = (g.N + kGN - 1) / kGN;
    int64_t tile = id % (mt * nt), bz = id / (mt * nt);
    if (g.ks % 8 == 0) {
        bz = (id & 7) + 8 * ((id >> 3) / (mt * nt));
        tile = (id >> 3) % (mt * nt);
    }
    const int64_t bx = tile % mt, by = tile / mt;
    const int64_t m0 = bx * kGM, n0 = by * kGN;
    const int64_t kb = bz * g.kchunk, ke = min(g.K, kb + g.kchunk);
    fx4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = fx4{0.0f, 0.0f, 0.0f, 0.0f};
    // the epilogue's own operands (z for EPI_DSILU and the inputs of the layer-1 sums) are loaded
    // before the main loop, so that their latency overlaps the staging
    fx4 pre[2][2];
    float xr[2][BP_MLP_NIN];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
        const int64_t m = m0 + 32 * wm + 16 * bi + (lane & 15);
#pragma unroll
        for (int q = 0; q < BP_MLP_NIN; ++q)
            xr[bi][q] = (EPI == EPI_DSILU && g.xs && m < g.M) ? g.xs[m * BP_MLP_IN + q] : 0.0f;
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            const int64_t n = n0 + 32 * wn + 16 * bj + 4 * (lane >> 4);
            const bool ok = m < g.M && n < g.N;
            pre[bi][bj] = fx4{0.0f, 0.0f, 0.0f, 0.0f};
            if (EPI == EPI_DSILU && ok) pre[bi][bj] = *(const fx4 *)(g.Z + m * g.ldz + n);
            if ((EPI == EPI_BIAS_SILU || EPI == EPI_BIAS) && ok)
                pre[bi][bj] = fx4{g.bias[n], g.bias[n + 1], g.bias[n + 2], g.bias[n + 3]};
            // a bias is the accumulators' starting value (as in the fused inference kernel)
            if (EPI == EPI_BIAS_SILU || EPI == EPI_BIAS) acc[bi][bj] = pre[bi][bj];
        }
    }
    for (int64_t k0 = kb; k0 < ke; k0 += kGKC) {
        const int64_t kend = min(ke, k0 + kGKC);
        if (kL1) stage_layer1(g, m0, by == 0, As, t);
        else if (kAK) stage_kmajor(g.A, g.a_m, m0, g.M, k0, kend, As, t);
        else stage_rmajor(g.A, g.a_k, m0, g.M, k0, kend, As, t);
        if (kBK1) stage_kmajor(g.B, g.b_n, n0, g.N, k0, kend, Bs, t);
        else stage_rmajor(g.B, g.b_k, n0, g.N, k0, kend, Bs, t);
        __syncthreads();
        const int steps = (int)((kend - k0 + kBK - 1) / kBK);
        // fragment rows of this lane and their swizzles
        const int ra0 = 32 * wm + (lane & 15), rb0 = 32 * wn + (lane & 15);
        const int sa[2] = {swz(ra0), swz(ra0 + 16)}, sb[2] = {swz(rb0), swz(rb0 + 16)};
        for (int ks = 0; ks < steps; ++ks) {
            const int grp = (lane >> 4) + 4 * ks;   // 16-byte group of k 32 ks + 8 (lane / 16)
            bf16x8 af[2], bfr[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                af[i] = *(const bf16x8 *)&As[ra0 + 16 * i][(grp ^ sa[i]) << 3];
                bfr[i] = *(const bf16x8 *)&Bs[rb0 + 16 * i][(grp ^ sb[i]) << 3];
            }
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = mfma32(bfr[bj], af[bi], acc[bi][bj]);
        }
        __syncthreads();
    }
    // epilogue: acc[bi][bj][j] is row m0 + 32 wm + 16 bi + lane % 16, column n0 + 32 wn + 16 bj + 4 (lane / 16) + j
    float csum[2][4][1 + BP_MLP_NIN];   // EPI_DSILU column sums over this lane's two rows
    const int ns = g.xs ? 1 + BP_MLP_NIN : 1;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
        const int64_t m = m0 + 32 * wm + 16 * bi + (lane & 15);
        const bool mok = m < g.M;
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            const int64_t n = n0 + 32 * wn + 16 * bj + 4 * (lane >> 4);
            const bool ok = mok && n < g.N;   // N % 8 == 0: a group of four is all in or all out
            const fx4 v = acc[bi][bj];
            if (EPI == EPI_BIAS_SILU) {
                if (!ok) continue;
                const fx4 z = v;
                if (g.Z) *(fx4 *)(g.Z + m * g.ldz + n) = z;
                st_bf4(g.H + m * g.ldh + n, silu(z[0]), silu(z[1]), silu(z[2]), silu(z[3]));
            } else if (EPI == EPI_BIAS) {
                if (!ok) continue;
                *(fx4 *)(g.F + m * g.ldf + n) = v;
            } else if (EPI == EPI_DSILU) {
                fx4 d = fx4{0.0f, 0.0f, 0.0f, 0.0f};
                if (ok) {
                    const fx4 z = pre[bi][bj];
                    d = fx4{v[0] * dsilu(z[0]), v[1] * dsilu(z[1]), v[2] * dsilu(z[2]), v[3] * dsilu(z[3])};
                    if (g.F) *(fx4 *)(g.F + m * g.ldf + n) = d;
                    if (g.H) st_bf4(g.H + m * g.ldh + n, d[0], d[1], d[2], d[3]);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float prev0 = bi ? csum[bj][j][0] : 0.0f;
                    csum[bj][j][0] = prev0 + d[j];
#pragma unroll
                    for (int q = 0; q < BP_MLP_NIN; ++q) {
                        const float prev = bi ? csum[bj][j][1 + q] : 0.0f;
                        csum[bj][j][1 + q] = prev + d[j] * xr[bi][q];
                    }
                }
            } else {
                if (!ok) continue;
                *(fx4 *)(g.F + (bz * g.M + m) * g.N + n) = v;
            }
        }
    }
    if (EPI == EPI_DSILU && g.cs) {
        // per-column sums over the tile's 64 rows (fixed order: the two rows of a lane, a butterfly over
        // the 16 lanes of one column group, then the two row halves of the tile), written as the chunk
        // partial cs[(bx * ns + s) * N + n], s = 0 for the plain sum and 1 + q for the sum weighted by
        // input q
        float (*red)[1 + BP_MLP_NIN][kGN] = (float (*)[1 + BP_MLP_NIN][kGN])&As[0][0];   // [2][ns][64]
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                for (int s = 0; s < ns; ++s) {
                    float c = csum[bj][j][s];
#pragma unroll
                    for (int o = 1; o < 16; o <<= 1) c += __shfl_xor(c, o, 64);
                    if ((lane & 15) == 0) red[wm][s][32 * wn + 16 * bj + 4 * (lane >> 4) + j] = c;
                }
        __syncthreads();
        if (t < ns * kGN) {
            const int s = t / kGN, nl = t % kGN;
            if (n0 + nl < g.N) g.cs[(bx * ns + s) * g.N + n0 + nl] = red[0][s][nl] + red[1][s][nl];
        }
    }
}

template <int EPI, bool kAK, bool kBK1, bool kL1 = false>
__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint16_t As[kGM][kGLd];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kGN][kGLd];
    gemm_tile<EPI, kAK, kBK1, kL1>(g, blockIdx.x, As, Bs);
}

// Two independent products in one launch: blocks below nb0 take g0's tiles, the rest g1's.
template <int E0, bool A0, bool B0, int E1, bool A1, bool B1>
__global__ void __launch_bounds__(256) k_gemm_pair(GemmArgs g0, int64_t nb0, GemmArgs g1) {
    __shared__ __attribute__((aligned(16))) uint16_t As[kGM][kGLd];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kGN][kGLd];
    if ((int64_t)blockIdx.x < nb0) gemm_tile<E0, A0, B0>(g0, blockIdx.x, As, Bs);
    else gemm_tile<E1, A1, B1>(g1, blockIdx.x - nb0, As, Bs);
}

static bool al(const void *p, int bytes) { return ((uintptr_t)p % bytes) == 0; }

// Layout and alignment checks of one product; its tile count in *tiles.
static int check_gemm(int epi, const GemmArgs &g, int ksplit, int64_t *tiles) {
    if (g.M <= 0 || g.N <= 0 || g.K <= 0 || ksplit < 1 || g.ks != ksplit || g.kchunk <= 0 || (g.kchunk % kBK))
        return BP_E_ARG;
    if ((int64_t)ksplit * g.kchunk < g.K) return BP_E_ARG;
    const bool ak = g.a_k == 1, bk = g.b_k == 1;
    // 16-byte loads along the contiguous dimension of each operand
    if (ak ? (g.a_m % 8 || g.K % 8) : (g.a_m != 1 || g.a_k % 8 || g.M % 8)) return BP_E_ARG;
    if (bk ? (g.b_n % 8 || g.K % 8) : (g.b_n != 1 || g.b_k % 8)) return BP_E_ARG;
    if (g.N % 8 || !al(g.A, 16) || !al(g.B, 16)) return BP_E_ARG;
    // vector epilogue: four FP32 (16 bytes) or four BF16 (8 bytes) per lane
    if (epi == EPI_BIAS_SILU && (!g.bias || !g.H || !al(g.H, 8) || g.ldh % 4 || (g.Z && (!al(g.Z, 16) || g.ldz % 4))))
        return BP_E_ARG;
    if (epi == EPI_BIAS && (!g.bias || !g.F || !al(g.F, 16) || g.ldf % 4)) return BP_E_ARG;
    if (epi == EPI_DSILU && (!g.Z || !al(g.Z, 16) || g.ldz % 4 || (g.H && (!al(g.H, 8) || g.ldh % 4)) ||
                             (g.F && (!al(g.F, 16) || g.ldf % 4))))
        return BP_E_ARG;
    if (epi == EPI_PARTIAL && (!g.F || !al(g.F, 16))) return BP_E_ARG;
    if (g.xs && epi != EPI_DSILU) return BP_E_ARG;
    *tiles = ((g.M + kGM - 1) / kGM) * ((g.N + kGN - 1) / kGN) * ksplit;
    return *tiles > 0x7fffffffLL ? BP_E_OVERFLOW : BP_OK;
}

static int launch_gemm(int epi, const GemmArgs &g, int ksplit, hipStream_t s) {
    int64_t tiles = 0;
    const int r = check_gemm(epi, g, ksplit, &tiles);
    if (r) return r;
    const dim3 grid((unsigned)tiles);
    const bool ak = g.a_k == 1, bk = g.b_k == 1;
#define BP_GEMM_LAUNCH(E)                                                                                   \
    do {                                                                                                     \
        if (ak && bk) hipLaunchKernelGGL((k_gemm_bf16<E, true, true>), grid, dim3(256), 0, s, g);           \
        else if (ak) hipLaunchKernelGGL((k_gemm_bf16<E, true, false>), grid, dim3(256), 0, s, g);           \
        else if (bk) hipLaunchKernelGGL((k_gemm_bf16<E, false, true>), grid, dim3(256), 0, s, g);           \
        else hipLaunchKernelGGL((k_gemm_bf16<E, false, false>), grid, dim3(256), 0, s, g);                  \
    } while (0)
    switch (epi) {
        case EPI_BIAS_SILU: BP_GEMM_LAUNCH(EPI_BIAS_SILU); break;
        case EPI_BIAS: BP_GEMM_LAUNCH(EPI_BIAS); break;
        case EPI_DSILU: BP_GEMM_LAUNCH(EPI_DSILU); break;
        default: BP_GEMM_LAUNCH(EPI_PARTIAL); break;
    }
#undef BP_GEMM_LAUNCH
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

// A weight gradient (EPI_PARTIAL, both operands contiguous in m / n) and the data gradient of the
// layer below (EPI_DSILU, A contiguous in k, B in n) in one launch: the two read the same upstream
// gradient and are independent.
static int launch_wgrad_dgrad(const GemmArgs &gw, int ksplit, const GemmArgs &gd, hipStream_t s) {
    int64_t tw = 0, td = 0;
    int r = check_gemm(EPI_PARTIAL, gw, ksplit, &tw);
    if (r) return r;
    r = check_gemm(EPI_DSILU, gd, 1, &td);
    if (r) return r;
    if (gw.a_k == 1 || gw.b_k == 1 || gd.a_k != 1 || gd.b_k == 1) return BP_E_ARG;
    if (tw + td > 0x7fffffffLL) return BP_E_OVERFLOW;
    hipLaunchKernelGGL((k_gemm_pair<EPI_PARTIAL, false, false, EPI_DSILU, true, false>), dim3((unsigned)(tw + td)),
                       dim3(256), 0, s, gw, tw, gd);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

// Column sums of the output gradient dy (the b4 gradient, for bp_mlp_backward) in fixed order:
// block (bx, y) covers 64 columns and the rows [64 y, 64 y + 64); its four waves take every fourth
// row and are combined in wave order, giving the chunk partial part[y][c], which Adam and
// k_reduce_grad sum in chunk order.
constexpr int kRowChunk = 64;
__global__ __launch_bounds__(256) void k_colsum_part(int64_t n, int cols, const float *__restrict__ a,
                                                     float *__restrict__ part) {
    __shared__ float red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + lane;
    const int64_t m0 = (int64_t)blockIdx.y * kRowChunk, m1 = min(n, m0 + kRowChunk);
    float acc = 0.0f;
    if (c < cols)
        for (int64_t m = m0 + w; m < m1; m += 4) acc += a[m * cols + c];
    red[w][lane] = acc;
    __syncthreads();
    if (w == 0 && c < cols)
        part[(int64_t)blockIdx.y * cols + c] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}
__global__ void k_to_bf16(int64_t n, const float *__restrict__ a, uint16_t *__restrict__ b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = f2bf(a[i]);
}

__global__ void k_adam(int64_t n, float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, uint16_t *__restrict__ wb, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.0f - b1) * gi;
    float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi; v[i] = vi;
    float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wb[i] = f2bf(wi);
}

// parameter offsets in the flat parameter vector
struct Off { int64_t W1, b1, W2, b2, W3, b3, W4, b4, total; };
static Off offsets() {
    Off o;
    o.W1 = 0; o.b1 = o.W1 + BP_MLP_HID * BP_MLP_IN;
    o.W2 = o.b1 + BP_MLP_HID; o.b2 = o.W2 + BP_MLP_HID * BP_MLP_HID;
    o.W3 = o.b2 + BP_MLP_HID; o.b3 = o.W3 + BP_MLP_HID * BP_MLP_HID;
    o.W4 = o.b3 + BP_MLP_HID; o.b4 = o.W4 + BP_MLP_OUT * BP_MLP_HID;
    o.total = o.b4 + BP_MLP_OUT;
    return o;
}

// activation buffer layout (per sample): z1 z2 z3 (fp32) and h1 h2 h3 (bf16)
static size_t act_bytes(int64_t n) { return (size_t)n * BP_MLP_HID * (3 * 4 + 3 * 2) + 1024; }

}  // namespace bp

using namespace bp;

extern "C" int64_t bp_mlp_nparams(void) { return offsets().total; }
extern "C" size_t bp_mlp_act_bytes(int64_t n) { return n < 0 ? 0 : act_bytes(n); }

namespace bp {
// The forward pass in three launches: layers 1 and 2 (layer 1 made in layer 2's operand staging),
// 3 and 4.  Input row m is x[m], or x[train_row(seed, step, m, ndata)] if ndata > 0 (the drawn
// rows' first BP_MLP_NIN inputs then go to xb).
static int forward(const float *w, const uint16_t *wb, int64_t n, const float *x, int64_t ndata, uint64_t seed,
                   int64_t step, float *xb, void *act, float *y, hipStream_t s) {
    const Off o = offsets();
    float *Z1 = (float *)act, *Z2 = Z1 + n * BP_MLP_HID, *Z3 = Z2 + n * BP_MLP_HID;
    uint16_t *H1 = (uint16_t *)(Z3 + n * BP_MLP_HID), *H2 = H1 + n * BP_MLP_HID, *H3 = H2 + n * BP_MLP_HID;
    GemmArgs g = {};
    g.M = n; g.K = BP_MLP_HID; g.kchunk = BP_MLP_HID; g.ks = 1;   // K = 256: one chunk
    // hidden layers: A = h (row-major [n][256]), B(k, n') = W[n'][k]
    g.N = BP_MLP_HID; g.A = nullptr; g.a_m = BP_MLP_HID; g.a_k = 1; g.B = wb + o.W2; g.b_k = 1; g.b_n = BP_MLP_HID;
    g.bias = w + o.b2; g.Z = Z2; g.ldz = BP_MLP_HID; g.H = H2; g.ldh = BP_MLP_HID;
    g.x1 = x; g.W1 = w + o.W1; g.b1 = w + o.b1; g.Z1 = Z1; g.H1 = H1; g.xb = xb;
    g.ndata = ndata; g.seed = seed; g.step = step;
    int64_t tiles = 0;
    int r = check_gemm(EPI_BIAS_SILU, g, 1, &tiles);
    if (r) return r;
    if (!x || (ndata > 0 && !xb)) return BP_E_ARG;
    hipLaunchKernelGGL((k_gemm_bf16<EPI_BIAS_SILU, true, true, true>), dim3((unsigned)tiles), dim3(256), 0, s, g);
    if (hipGetLastError() != hipSuccess) return BP_E_HIP;
    g = GemmArgs{};
    g.M = n; g.K = BP_MLP_HID; g.kchunk = BP_MLP_HID; g.ks = 1;
    g.N = BP_MLP_HID; g.A = H2; g.a_m = BP_MLP_HID; g.a_k = 1; g.B = wb + o.W3; g.b_k = 1; g.b_n = BP_MLP_HID;
    g.bias = w + o.b3; g.Z = Z3; g.ldz = BP_MLP_HID; g.H = H3; g.ldh = BP_MLP_HID;
    r = launch_gemm(EPI_BIAS_SILU, g, 1, s);
    if (r) return r;
    g.N = BP_MLP_OUT; g.A = H3; g.B = wb + o.W4; g.bias = w + o.b4; g.F = y; g.ldf = BP_MLP_OUT; g.Z = nullptr;
    g.H = nullptr;
    return launch_gemm(EPI_BIAS, g, 1, s);
}

int mlp_forward_train(const float *w, const uint16_t *wb, int64_t n, int64_t ndata, uint64_t seed, int64_t step,
                      const float *xdata, float *xb, void *act, float *y, hipStream_t s) {
    if (n <= 0 || ndata <= 0 || !w || !wb || !xdata || !xb || !act || !y) return BP_E_ARG;
    if (((uintptr_t)xdata | (uintptr_t)xb | (uintptr_t)act | (uintptr_t)y | (uintptr_t)wb) & 15) return BP_E_ARG;
    return forward(w, wb, n, xdata, ndata, seed, step, xb, act, y, s);
}
}  // namespace bp

extern "C" int bp_mlp_forward(const float *w, const uint16_t *wb, int64_t n, const float *x, float *y, void *act,
                              void *stream) {
    if (n < 0 || !w || !wb || !x || !y || !act) return BP_E_ARG;
    if (n == 0) return BP_OK;
    if (((uintptr_t)y | (uintptr_t)act | (uintptr_t)wb) & 15) return BP_E_ARG;   // 16-byte vector access
    hipStream_t s = (hipStream_t)stream;
    prof_begin(BP_PROF_MLP_FWD, s);
    const int r = forward(w, wb, n, x, 0, 0, 0, nullptr, act, y, s);
    prof_end(BP_PROF_MLP_FWD, s);
    return r;
}

// ------------------------------------------------------------ fused inference --
// All four layers for a block of 128 rows in one kernel; activations never leave the CU (one
// 128 x 256 BF16 buffer in LDS, rewritten in place by each layer).  Each layer is computed
// transposed, out^T = W h^T: the weights are the MFMA A operand, read by each wavefront straight from
// memory (they stay in L2), and the activations are the B operand, read from LDS.  Each of the
// eight wavefronts owns two 16-feature output blocks of a hidden layer (2w, 2w + 1; w and w + 8 of
// the 9 output blocks) for all 128 rows, so no weight fragment is fetched twice within a workgroup;
// the fragments run kIPf k slices ahead of the MFMAs.  A lane's accumulator holds four consecutive
// features of one row, starting from the bias, and the epilogue writes them back as BF16 once every
// wavefront has read the layer's input.  The 66 KB of LDS and at most 128 registers per lane let
// two workgroups (sixteen wavefronts) share a CU, so that one wavefront's SiLU work overlaps
// another's MFMAs.  The k order of every sum is that of bp_mlp_forward, so the outputs are the same
// bit for bit.
constexpr int kIR = 128;                 // rows per workgroup
constexpr int kIRB = kIR / 16;           // 16-row blocks
constexpr int kIW = 8;                   // wavefronts per workgroup
constexpr int kIOB = BP_MLP_HID / 16 / kIW;   // output blocks per wavefront in a hidden layer (2)
constexpr int kIK = 32;                  // k per MFMA
constexpr int kIKB = BP_MLP_HID / kIK;   // k slices of a layer
constexpr int kIPf = 2;                  // k slices of weight fragments in flight
constexpr int kIALd = BP_MLP_HID + 8;    // LDS row stride of the activations (bf16)
constexpr int kIOutB = BP_MLP_OUT / 16;  // output blocks of the last layer
static_assert(kIKB % kIPf == 0 && kIOutB <= 2 * kIW, "prefetch ring and output-block assignment");

// acc[rb][j] += sum_k W[16 ob_j + .][k] h[16 rb + .][k] for the wavefront's blocks ob_j = ob0 + ostride j,
// j < NOB; W is [.][256] BF16 row-major.  (MFMAs ignore the execution mask, so a block count below
// kIOB is a separate instance rather than a masked one.)
template <int NOB>
__device__ inline void infer_layer(const uint16_t *__restrict__ W, int ob0, int ostride,
                                   const uint16_t *__restrict__ acts, fx4 (&acc)[kIRB][kIOB], int lane) {
    const uint16_t *wbase = W + (int64_t)__builtin_amdgcn_readfirstlane(16 * ob0) * BP_MLP_HID;
    const int jstride = 16 * ostride * BP_MLP_HID, loff = (lane & 15) * BP_MLP_HID + 8 * (lane >> 4);
    bf16x8 pf[kIPf][NOB];
#pragma unroll
    for (int p = 0; p < kIPf; ++p)
#pragma unroll
        for (int j = 0; j < NOB; ++j) pf[p][j] = *(const bf16x8 *)(wbase + j * jstride + loff + kIK * p);
    const uint16_t *bsrc = acts + (lane & 15) * kIALd + 8 * (lane >> 4);
#pragma unroll
    for (int kb = 0; kb < kIKB; ++kb) {
        bf16x8 a[NOB];
#pragma unroll
        for (int j = 0; j < NOB; ++j) a[j] = pf[kb % kIPf][j];
        if (kb + kIPf < kIKB)
#pragma unroll
            for (int j = 0; j < NOB; ++j)
                pf[kb % kIPf][j] = *(const bf16x8 *)(wbase + j * jstride + loff + kIK * (kb + kIPf));
#pragma unroll
        for (int rb = 0; rb < kIRB; ++rb) {
            const bf16x8 b = *(const bf16x8 *)(bsrc + 16 * rb * kIALd + kIK * kb);
#pragma unroll
            for (int j = 0; j < NOB; ++j) acc[rb][j] = mfma32(a[j], b, acc[rb][j]);
        }
    }
}

__global__ void __launch_bounds__(64 * kIW) __attribute__((amdgpu_waves_per_eu(4))) k_mlp_infer(int64_t n, const float *__restrict__ w,
                                                           const uint16_t *__restrict__ wb,
                                                           const float *__restrict__ x, float *__restrict__ y,
                                                           int64_t oW1, int64_t ob1, int64_t oW2, int64_t ob2,
                                                           int64_t oW3, int64_t ob3, int64_t oW4, int64_t ob4) {
    __shared__ __attribute__((aligned(16))) uint16_t acts[kIR * kIALd];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * kIR;
    // layer 1 (FP32): thread t makes features 4 (t % 64) .. + 3 of rows t / 64 + kIW i
    {
        const int fq = 4 * lane;
        float bv[4], wq[4][BP_MLP_NIN];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            bv[j] = w[ob1 + fq + j];
#pragma unroll
            for (int q = 0; q < BP_MLP_NIN; ++q) wq[j][q] = w[oW1 + (fq + j) * BP_MLP_IN + q];
        }
        // the wavefront's kIR / kIW rows of inputs in one load: lane 3 i + q holds x[row i][q]
        static_assert(BP_MLP_NIN * (kIR / kIW) <= 64, "one input per lane");
        float xl = 0.0f;
        {
            const int i = lane / BP_MLP_NIN, q = lane - BP_MLP_NIN * i;
            const int64_t row = row0 + wv + kIW * i;
            if (i < kIR / kIW && row < n) xl = x[row * BP_MLP_IN + q];
        }
#pragma unroll
        for (int i = 0; i < kIR / kIW; ++i) {
            const int r = wv + kIW * i;   // one row per wavefront
            float xr[BP_MLP_NIN];
#pragma unroll
            for (int q = 0; q < BP_MLP_NIN; ++q)
                xr[q] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(xl), BP_MLP_NIN * i + q));
            float h[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) h[j] = silu(layer1_z(bv[j], wq[j], xr));
            *(sx4 *)(acts + r * kIALd + fq) = pack_bf4(h[0], h[1], h[2], h[3]);
        }
    }
    __syncthreads();
    // hidden layers 2 and 3
    const int frow = lane & 15, fcol = 4 * (lane >> 4);   // a lane's row in a 16-row block, feature in a 16-block
    fx4 acc[kIRB][kIOB];
    for (int layer = 0; layer < 2; ++layer) {
        const float *bias = w + (layer == 0 ? ob2 : ob3);
#pragma unroll
        for (int j = 0; j < kIOB; ++j) {
            const int f = 16 * (kIOB * wv + j) + fcol;
            const fx4 bb = fx4{bias[f], bias[f + 1], bias[f + 2], bias[f + 3]};
#pragma unroll
            for (int rb = 0; rb < kIRB; ++rb) acc[rb][j] = bb;
        }
        infer_layer<kIOB>(wb + (layer == 0 ? oW2 : oW3), kIOB * wv, 1, acts, acc, lane);
        __syncthreads();   // every wavefront has read the layer's input
#pragma unroll
        for (int rb = 0; rb < kIRB; ++rb)
#pragma unroll
            for (int j = 0; j < kIOB; ++j) {
                const fx4 z = acc[rb][j];
                *(sx4 *)(acts + (16 * rb + frow) * kIALd + 16 * (kIOB * wv + j) + fcol) =
                    pack_bf4(silu(z[0]), silu(z[1]), silu(z[2]), silu(z[3]));
            }
        __syncthreads();
    }
    // output layer: blocks wv and wv + kIW (< 9)
    const int nob = __builtin_amdgcn_readfirstlane((wv + kIW < kIOutB) ? 2 : 1);
#pragma unroll
    for (int j = 0; j < kIOB; ++j) {
        const int f = 16 * (wv + kIW * j) + fcol;
        const fx4 bb = j < nob ? fx4{w[ob4 + f], w[ob4 + f + 1], w[ob4 + f + 2], w[ob4 + f + 3]}
                               : fx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int rb = 0; rb < kIRB; ++rb) acc[rb][j] = bb;
    }
    if (nob == 2) infer_layer<2>(wb + oW4, wv, kIW, acts, acc, lane);
    else infer_layer<1>(wb + oW4, wv, kIW, acts, acc, lane);
#pragma unroll
    for (int rb = 0; rb < kIRB; ++rb) {
        const int64_t row = row0 + 16 * rb + frow;
        if (row >= n) continue;
#pragma unroll
        for (int j = 0; j < kIOB; ++j)
            if (j < nob) *(fx4 *)(y + row * BP_MLP_OUT + 16 * (wv + kIW * j) + fcol) = acc[rb][j];
    }
}

extern "C" int bp_mlp_infer(const float *w, const uint16_t *wb, int64_t n, const float *x, float *y, void *stream) {
    if (n < 0 || !w || !wb || !x || !y) return BP_E_ARG;
    if (n == 0) return BP_OK;
    if ((((uintptr_t)y) & 15) || (((uintptr_t)wb) & 15)) return BP_E_ARG;   // 16-byte vector access
    const int64_t blocks = (n + kIR - 1) / kIR;
    if (blocks > 0x7fffffffLL) return BP_E_OVERFLOW;
    hipStream_t s = (hipStream_t)stream;
    Off o = offsets();
    prof_begin(BP_PROF_MLP_FWD, s);
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)blocks), dim3(64 * kIW), 0, s, n, w, wb, x, y, o.W1, o.b1, o.W2, o.b2,
                       o.W3, o.b3, o.W4, o.b4);
    prof_end(BP_PROF_MLP_FWD, s);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

// split-K factor of the weight-gradient products (K = batch): slices of at most 256 rows, one LDS
// stage each, up to 64 slices
static int wgrad_splits(int64_t n) {
    int64_t ks = (n + kGKC - 1) / kGKC;
    return (int)(ks < 1 ? 1 : ks > 64 ? 64 : ks);
}

// The gradient as partial sums that the consumer reduces in a fixed order (GradParts): all of them
// coexist, so one kernel reduces every parameter.
static_assert(kRowChunk == kGM, "the data-gradient epilogue leaves one column partial per 64-row tile");
static int64_t nchunks(int64_t n) { return (n + kRowChunk - 1) / kRowChunk; }

static size_t part_floats(int64_t n) {
    const int64_t ks = wgrad_splits(n), nc = nchunks(n);
    return (size_t)(ks * (BP_MLP_OUT + 2 * BP_MLP_HID) * BP_MLP_HID +
                    nc * (BP_MLP_OUT + 2 * BP_MLP_HID + (1 + BP_MLP_NIN) * BP_MLP_HID)) + 64;
}

// the partials' places in a workspace of part_floats(n) floats
static GradParts parts_layout(float *part, int64_t n) {
    GradParts P;
    P.ks = wgrad_splits(n);
    P.nchunk = (int)nchunks(n);
    float *q = part;
    P.w4 = q; q += (int64_t)P.ks * BP_MLP_OUT * BP_MLP_HID;
    P.w3 = q; q += (int64_t)P.ks * BP_MLP_HID * BP_MLP_HID;
    P.w2 = q; q += (int64_t)P.ks * BP_MLP_HID * BP_MLP_HID;
    P.b4 = q; q += (int64_t)P.nchunk * BP_MLP_OUT;
    P.b3 = q; q += (int64_t)P.nchunk * BP_MLP_HID;
    P.b2 = q; q += (int64_t)P.nchunk * BP_MLP_HID;
    P.l1 = q;
    return P;
}

// sum_{q < count} p[q * stride] from zero in q order; the loads go out eight at a time ahead of the
// adds, so a thread waits on memory count / 8 times rather than count times
__device__ inline float sum_in_order(const float *__restrict__ p, int64_t stride, int count) {
    float s = 0.0f;
    int q = 0;
    for (; q + 8 <= count; q += 8) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = p[(int64_t)(q + j) * stride];
#pragma unroll
        for (int j = 0; j < 8; ++j) s += v[j];
    }
    for (; q < count; ++q) s += p[(int64_t)q * stride];
    return s;
}

// Gradient of parameter p from the partials, each group summed in slice / chunk order from zero.
__device__ inline float grad_of(const GradParts &P, const Off &o, int64_t p) {
    constexpr int64_t kHH = (int64_t)BP_MLP_HID * BP_MLP_HID, kOH = (int64_t)BP_MLP_OUT * BP_MLP_HID;
    if (p >= o.b4) return sum_in_order(P.b4 + (p - o.b4), BP_MLP_OUT, P.nchunk);
    if (p >= o.W4) return sum_in_order(P.w4 + (p - o.W4), kOH, P.ks);
    if (p >= o.b3) return sum_in_order(P.b3 + (p - o.b3), BP_MLP_HID, P.nchunk);
    if (p >= o.W3) return sum_in_order(P.w3 + (p - o.W3), kHH, P.ks);
    if (p >= o.b2) return sum_in_order(P.b2 + (p - o.b2), BP_MLP_HID, P.nchunk);
    if (p >= o.W2) return sum_in_order(P.w2 + (p - o.W2), kHH, P.ks);
    constexpr int64_t kL1 = (int64_t)(1 + BP_MLP_NIN) * BP_MLP_HID;   // one chunk of the layer-1 sums
    if (p >= o.b1) return sum_in_order(P.l1 + (p - o.b1), kL1, P.nchunk);
    const int64_t row = p / BP_MLP_IN, k = p - row * BP_MLP_IN;   // W1[row][k]; inputs past NIN are padding
    return k < BP_MLP_NIN ? sum_in_order(P.l1 + (1 + k) * BP_MLP_HID + row, kL1, P.nchunk) : 0.0f;
}

__global__ void k_reduce_grad(GradParts P, Off o, float *__restrict__ grad) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < o.total) grad[p] = grad_of(P, o, p);
}

// one Adam step straight from the partials (the reduction of k_reduce_grad, then the update of
// k_adam); the gradient is also written to g
__global__ void k_adam_parts(GradParts P, Off o, float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                             float *__restrict__ g, uint16_t *__restrict__ wb, float lr, float b1, float b2, float eps,
                             float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= o.total) return;
    const float gi = grad_of(P, o, i);
    g[i] = gi;
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi; v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wb[i] = f2bf(wi);
}

extern "C" size_t bp_mlp_backward_ws_bytes(int64_t n) {
    if (n <= 0) return 0;
    return ((size_t)n * BP_MLP_OUT * 2 + 255) / 256 * 256 + 2 * (((size_t)n * BP_MLP_HID * 2 + 255) / 256 * 256) +
           part_floats(n) * 4 + 1024;
}

namespace bp {
// workspace: G4 [n][144] bf16, Gb and Gc [n][256] bf16 (the upstream gradients of layers 3 and 2),
// then the partials
struct BwdWs {
    uint16_t *G4, *Gb, *Gc;
    float *part;
};
static bool bwd_ws(void *ws, size_t ws_bytes, int64_t n, BwdWs *B) {
    Arena A(ws, ws_bytes);
    B->G4 = A.take<uint16_t>(n * BP_MLP_OUT);
    B->Gb = A.take<uint16_t>(n * BP_MLP_HID);
    B->Gc = A.take<uint16_t>(n * BP_MLP_HID);
    B->part = A.take<float>((int64_t)part_floats(n));
    return A.fits() && ws_bytes >= bp_mlp_backward_ws_bytes(n);
}

int mlp_backward_layout(void *ws, size_t ws_bytes, int64_t n, uint16_t **g4, GradParts *P) {
    if (n <= 0 || !ws || ((uintptr_t)ws % 256)) return BP_E_ARG;
    BwdWs B;
    if (!bwd_ws(ws, ws_bytes, n, &B)) return BP_E_WORKSPACE;
    *g4 = B.G4;
    *P = parts_layout(B.part, n);
    return BP_OK;
}

// Three launches, each the weight gradient of one layer beside the data gradient of the layer below
// (whose epilogue also leaves the bias partials, and for layer 1 the input-weighted sums).
int mlp_backward_g4(const uint16_t *wb, int64_t n, const float *x, const void *act, void *ws, size_t ws_bytes,
                    hipStream_t s) {
    if (n <= 0 || !wb || !x || !act || !ws) return BP_E_ARG;
    if ((((uintptr_t)x | (uintptr_t)act | (uintptr_t)wb) & 15) || ((uintptr_t)ws % 256)) return BP_E_ARG;
    BwdWs B;
    if (!bwd_ws(ws, ws_bytes, n, &B)) return BP_E_WORKSPACE;
    const GradParts P = parts_layout(B.part, n);
    const Off o = offsets();
    const float *Z1 = (const float *)act, *Z2 = Z1 + n * BP_MLP_HID, *Z3 = Z2 + n * BP_MLP_HID;
    const uint16_t *H1 = (const uint16_t *)(Z3 + n * BP_MLP_HID), *H2 = H1 + n * BP_MLP_HID, *H3 = H2 + n * BP_MLP_HID;
    const int ks = P.ks;
    const int64_t kchunk = (((n + ks - 1) / ks + kBK - 1) / kBK) * kBK;
    // dW = G^T h over the batch in ks split-K slices: A(m = o, k = s) = G[s][o], B(k = s, n = i) = h[s][i]
    auto wgrad = [&](const uint16_t *Gt, int64_t ldg, int64_t rows, const uint16_t *Hin, const float *dst) {
        GemmArgs g = {};
        g.M = rows; g.N = BP_MLP_HID; g.K = n; g.kchunk = kchunk; g.ks = ks;
        g.A = Gt; g.a_m = 1; g.a_k = ldg;
        g.B = Hin; g.b_k = BP_MLP_HID; g.b_n = 1;
        g.F = (float *)dst;
        return g;
    };
    // d = (G W) * silu'(z): A(s, o) = G[s][o], B(o, i) = W[o][i]; column sums into cs
    auto dgrad = [&](const uint16_t *Gin, int64_t kdim, const uint16_t *W, const float *Z, uint16_t *Gout,
                     const float *cs, const float *xs) {
        GemmArgs g = {};
        g.M = n; g.N = BP_MLP_HID; g.K = kdim; g.kchunk = ((kdim + kBK - 1) / kBK) * kBK; g.ks = 1;
        g.A = Gin; g.a_m = kdim; g.a_k = 1;
        g.B = W; g.b_k = BP_MLP_HID; g.b_n = 1;
        g.Z = (float *)Z; g.ldz = BP_MLP_HID; g.H = Gout; g.ldh = BP_MLP_HID;
        g.cs = (float *)cs; g.xs = xs;
        return g;
    };
    int r = launch_wgrad_dgrad(wgrad(B.G4, BP_MLP_OUT, BP_MLP_OUT, H3, P.w4), ks,
                               dgrad(B.G4, BP_MLP_OUT, wb + o.W4, Z3, B.Gb, P.b3, nullptr), s);
    if (r) return r;
    r = launch_wgrad_dgrad(wgrad(B.Gb, BP_MLP_HID, BP_MLP_HID, H2, P.w3), ks,
                           dgrad(B.Gb, BP_MLP_HID, wb + o.W3, Z2, B.Gc, P.b2, nullptr), s);
    if (r) return r;
    // layer 1: only the sums of d1 are needed (db1 and dW1), d1 itself is not stored
    return launch_wgrad_dgrad(wgrad(B.Gc, BP_MLP_HID, BP_MLP_HID, H1, P.w2), ks,
                              dgrad(B.Gc, BP_MLP_HID, wb + o.W2, Z1, nullptr, P.l1, x), s);
}

// The backward pass up to the partials (workspace as bp_mlp_backward); *P receives their places.
int mlp_backward_parts(const float *w, const uint16_t *wb, int64_t n, const float *x, const void *act,
                       const float *dy, GradParts *P, void *ws, size_t ws_bytes, hipStream_t s) {
    if (n <= 0 || !w || !wb || !x || !act || !dy || !ws) return BP_E_ARG;
    uint16_t *G4 = nullptr;
    int r = mlp_backward_layout(ws, ws_bytes, n, &G4, P);
    if (r) return r;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n * BP_MLP_OUT + 255) / 256)), dim3(256), 0, s, n * BP_MLP_OUT, dy,
                       G4);
    hipLaunchKernelGGL(k_colsum_part, dim3((BP_MLP_OUT + 63) / 64, P->nchunk), dim3(256), 0, s, n, BP_MLP_OUT, dy,
                       (float *)P->b4);
    if (hipGetLastError() != hipSuccess) return BP_E_HIP;
    return mlp_backward_g4(wb, n, x, act, ws, ws_bytes, s);
}

// Adam from the partials of mlp_backward_parts, the bias corrections for `step` (>= 1).
int mlp_adam_parts(const GradParts &P, float *w, float *m, float *v, float *g, uint16_t *wb, float lr, float b1,
                   float b2, float eps, int64_t step, hipStream_t s) {
    const Off o = offsets();
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam_parts, dim3((unsigned)((o.total + 255) / 256)), dim3(256), 0, s, P, o, w, m, v, g, wb, lr,
                       b1, b2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}
}  // namespace bp

extern "C" int bp_mlp_backward(const float *w, const uint16_t *wb, int64_t n, const float *x, const void *act,
                               const float *dy, float *grad, void *ws, size_t ws_bytes, void *stream) {
    if (n <= 0 || !w || !wb || !x || !act || !dy || !grad || !ws) return BP_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    GradParts P;
    prof_begin(BP_PROF_MLP_BWD, s);
    int r = mlp_backward_parts(w, wb, n, x, act, dy, &P, ws, ws_bytes, s);
    if (r) return r;
    const Off o = offsets();
    hipLaunchKernelGGL(k_reduce_grad, dim3((unsigned)((o.total + 255) / 256)), dim3(256), 0, s, P, o, grad);
    prof_end(BP_PROF_MLP_BWD, s);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

extern "C" int bp_mlp_adam(int64_t np, float *w, float *m, float *v, const float *g, uint16_t *wb, float lr, float b1,
                           float b2, float eps, int64_t step, void *stream) {
    if (np <= 0 || !w || !m || !v || !g || !wb || step < 1) return BP_E_ARG;
    float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, (hipStream_t)stream, np, w, m, v, g,
                       wb, lr, b1, b2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

extern "C" int bp_mlp_to_bf16(int64_t np, const float *w, uint16_t *wb, void *stream) {
    if (np <= 0 || !w || !wb) return BP_E_ARG;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, (hipStream_t)stream, np, w, wb);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}
