// K10-K12: the profile-table surrogate network, forward, backward and Adam.
//
// Network (inputs normalised (log10 M, ln c, z)):
//   z1 = W1 x + b1                       FP32 (3 inputs: VALU)
//   h1 = bf16(silu(z1))
//   z2 = W2 h1 + b2, h2 = bf16(silu(z2)) BF16 MFMA, FP32 accumulation
//   z3 = W3 h2 + b3, h3 = bf16(silu(z3))
//   y  = W4 h3 + b4                      FP32 output
// The hidden-layer products run on gfx950's v_mfma_f32_16x16x32_bf16 (a 16x16
// block over 32 k per instruction): a workgroup computes a 128x64 output tile
// with four wavefronts (2x4 blocks of 16x16 each), staging 32-wide k slices of
// both operands in LDS per K step.  Weight
// gradients reduce over the batch with split-K partial tiles summed in a
// fixed order, so training is deterministic.
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

// round-to-nearest-even FP32 -> BF16 (gfx950 converts in hardware, v_cvt_pk_bf16_f32)
__device__ inline uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
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
};

// 128x64 output tile per workgroup; wavefront w owns rows 32w..32w+31 (2x4 blocks of 16x16).
// K advances 32 at a time, one MFMA per block; both operands are staged in LDS with k contiguous
// (B transposed), so each MFMA fragment is a single 16-byte LDS read.  All vectorised operand dimensions in this
// library are multiples of 8 (K, the 256/144 layer widths); the batch dimension M is guarded per row.
constexpr int kBM = 128, kBN = 64, kBK = 32, kLdk = kBK + 8;   // +8 bf16 of padding per row

typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

template <int EPI>
__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint16_t As[kBM][kLdk];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kBN][kLdk];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t m0 = (int64_t)blockIdx.x * kBM, n0 = (int64_t)blockIdx.y * kBN;
    const int64_t kb = (int64_t)blockIdx.z * g.kchunk;
    const int64_t ke = min(g.K, kb + g.kchunk);
    fx4 acc[2][4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 4; ++b) acc[a][b] = fx4{0.0f, 0.0f, 0.0f, 0.0f};
    const u16x8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t k0 = kb; k0 < ke; k0 += kBK) {
        // ---- stage A tile (128 x 32) into As[m][k]
        if (g.a_k == 1) {
            // rows contiguous in k: thread t loads 16 elements of row t/2
            int am = t >> 1, ak = (t & 1) * 16;
            int64_t gm = m0 + am;
            for (int h = 0; h < 2; ++h) {
                int64_t gk = k0 + ak + 8 * h;
                u16x8 v = zero8;
                if (gm < g.M && gk < ke) v = *(const u16x8 *)(g.A + gm * g.a_m + gk);
                *(u16x8 *)&As[am][ak + 8 * h] = v;
            }
        } else {
            // columns contiguous in m (a_m == 1): thread t loads 8 m-values at k = t/8 ... twice
            for (int h = 0; h < 2; ++h) {
                int e = t + 256 * h;
                int ak = e >> 4, am = (e & 15) * 8;
                int64_t gk = k0 + ak, gm = m0 + am;
                u16x8 v = zero8;
                if (gk < ke && gm + 7 < g.M) v = *(const u16x8 *)(g.A + gk * g.a_k + gm);
                else if (gk < ke)
                    for (int j = 0; j < 8; ++j) v[j] = (gm + j < g.M) ? g.A[gk * g.a_k + gm + j] : (uint16_t)0;
                for (int j = 0; j < 8; ++j) As[am + j][ak] = v[j];
            }
        }
        // ---- stage B tile (32 x 64) into Bs[n][k]
        if (g.b_k == 1) {
            int bn = t >> 2, bk = (t & 3) * 8;
            int64_t gn = n0 + bn, gk = k0 + bk;
            u16x8 v = zero8;
            if (gn < g.N && gk < ke) v = *(const u16x8 *)(g.B + gn * g.b_n + gk);
            *(u16x8 *)&Bs[bn][bk] = v;
        } else {
            int bk = t >> 3, bn = (t & 7) * 8;
            int64_t gk = k0 + bk, gn = n0 + bn;
            u16x8 v = zero8;
            if (gk < ke && gn < g.N) v = *(const u16x8 *)(g.B + gk * g.b_k + gn);
            for (int j = 0; j < 8; ++j) Bs[bn + j][bk] = v[j];
        }
        __syncthreads();
        {
            static_assert(kBK == 32, "one 16x16x32 MFMA per block and K step");
            bf16x8 af[2], bfr[4];
            for (int bi = 0; bi < 2; ++bi)
                af[bi] = *(const bf16x8 *)&As[32 * w + 16 * bi + (lane & 15)][8 * (lane >> 4)];
            for (int bj = 0; bj < 4; ++bj)
                bfr[bj] = *(const bf16x8 *)&Bs[16 * bj + (lane & 15)][8 * (lane >> 4)];
            for (int bi = 0; bi < 2; ++bi)
                for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mfma32(af[bi], bfr[bj], acc[bi][bj]);
        }
        __syncthreads();
    }
    // epilogue: lane holds D[4*(lane>>4)+j][lane&15] of each 16x16 block
    for (int bi = 0; bi < 2; ++bi)
        for (int bj = 0; bj < 4; ++bj)
            for (int j = 0; j < 4; ++j) {
                int64_t m = m0 + 32 * w + 16 * bi + 4 * (lane >> 4) + j;
                int64_t n = n0 + 16 * bj + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                float v = acc[bi][bj][j];
                if (EPI == EPI_BIAS_SILU) {
                    float z = v + g.bias[n];
                    if (g.Z) g.Z[m * g.ldz + n] = z;
                    g.H[m * g.ldh + n] = f2bf(silu(z));
                } else if (EPI == EPI_BIAS) {
                    g.F[m * g.ldf + n] = v + g.bias[n];
                } else if (EPI == EPI_DSILU) {
                    float d = v * dsilu(g.Z[m * g.ldz + n]);
                    if (g.F) g.F[m * g.ldf + n] = d;
                    g.H[m * g.ldh + n] = f2bf(d);
                } else {
                    g.F[(int64_t)blockIdx.z * g.M * g.N + m * g.N + n] = v;
                }
            }
}

static int launch_gemm(int epi, const GemmArgs &g, int ksplit, hipStream_t s) {
    if ((g.M + kBM - 1) / kBM > 0x7fffffffLL) return BP_E_OVERFLOW;
    // the vectorised staging needs 16-byte aligned rows along the contiguous dimension
    if ((g.a_k == 1 && (g.a_m % 8)) || (g.a_k != 1 && (g.a_k % 8 || g.a_m != 1)) || (g.b_k == 1 && (g.b_n % 8)) ||
        (g.b_k != 1 && (g.b_k % 8 || g.b_n != 1)) || (g.kchunk % kBK) ||
        ((g.a_k == 1 || g.b_k == 1) && (g.K % 8)) || (g.N % 8))
        return BP_E_ARG;
    dim3 grid((unsigned)((g.M + kBM - 1) / kBM), (unsigned)((g.N + kBN - 1) / kBN), (unsigned)ksplit);
    switch (epi) {
        case EPI_BIAS_SILU: hipLaunchKernelGGL(k_gemm_bf16<EPI_BIAS_SILU>, grid, dim3(256), 0, s, g); break;
        case EPI_BIAS: hipLaunchKernelGGL(k_gemm_bf16<EPI_BIAS>, grid, dim3(256), 0, s, g); break;
        case EPI_DSILU: hipLaunchKernelGGL(k_gemm_bf16<EPI_DSILU>, grid, dim3(256), 0, s, g); break;
        default: hipLaunchKernelGGL(k_gemm_bf16<EPI_PARTIAL>, grid, dim3(256), 0, s, g); break;
    }
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

// first layer in FP32: z1 = W1 x + b1, h1 = bf16(silu(z1)); x has BP_MLP_IN columns (only BP_MLP_NIN used)
__global__ void k_layer1(int64_t n, const float *__restrict__ W1, const float *__restrict__ b1,
                         const float *__restrict__ x, float *__restrict__ Z1, uint16_t *__restrict__ H1) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * BP_MLP_HID) return;
    int64_t m = e / BP_MLP_HID;
    int o = (int)(e % BP_MLP_HID);
    float z = b1[o];
    for (int k = 0; k < BP_MLP_NIN; ++k) z += W1[o * BP_MLP_IN + k] * x[m * BP_MLP_IN + k];
    if (Z1) Z1[e] = z;
    H1[e] = f2bf(silu(z));
}

// sum over split-K partials in fixed order: out[i] = sum_s part[s][i]
// Batch reductions in two fixed-order stages.  Stage 1: block (bx, y) covers 64 columns and the rows
// [64 y, 64 y + 64); its four waves take every fourth row and are combined in wave order, giving
// part[y][j][c] = sum_m a[m][c] * (j == 0 ? 1 : x[m][j - 1]).  Stage 2 sums the chunks in order.
constexpr int kRowChunk = 64;
template <int kSums>
__global__ __launch_bounds__(256) void k_colsum_part(int64_t n, int cols, const float *__restrict__ a,
                                                     const float *__restrict__ x, float *__restrict__ part) {
    __shared__ float red[4][kSums][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + lane;
    const int64_t m0 = (int64_t)blockIdx.y * kRowChunk, m1 = min(n, m0 + kRowChunk);
    float acc[kSums];
#pragma unroll
    for (int j = 0; j < kSums; ++j) acc[j] = 0.0f;
    if (c < cols)
        for (int64_t m = m0 + w; m < m1; m += 4) {
            float v = a[m * cols + c];
            acc[0] += v;
#pragma unroll
            for (int j = 1; j < kSums; ++j) acc[j] += v * x[m * BP_MLP_IN + j - 1];
        }
#pragma unroll
    for (int j = 0; j < kSums; ++j) red[w][j][lane] = acc[j];
    __syncthreads();
    if (w == 0 && c < cols)
#pragma unroll
        for (int j = 0; j < kSums; ++j)
            part[((int64_t)blockIdx.y * kSums + j) * cols + c] =
                ((red[0][j][lane] + red[1][j][lane]) + red[2][j][lane]) + red[3][j][lane];
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

extern "C" int bp_mlp_forward(const float *w, const uint16_t *wb, int64_t n, const float *x, float *y, void *act,
                              void *stream) {
    if (n < 0 || !w || !wb || !x || !y || !act) return BP_E_ARG;
    if (n == 0) return BP_OK;
    hipStream_t s = (hipStream_t)stream;
    Off o = offsets();
    float *Z1 = (float *)act, *Z2 = Z1 + n * BP_MLP_HID, *Z3 = Z2 + n * BP_MLP_HID;
    uint16_t *H1 = (uint16_t *)(Z3 + n * BP_MLP_HID), *H2 = H1 + n * BP_MLP_HID, *H3 = H2 + n * BP_MLP_HID;
    prof_begin(BP_PROF_MLP_FWD, s);
    int64_t e = n * BP_MLP_HID;
    hipLaunchKernelGGL(k_layer1, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, s, n, w + o.W1, w + o.b1, x, Z1, H1);
    GemmArgs g = {};
    g.M = n; g.K = BP_MLP_HID; g.kchunk = BP_MLP_HID;   // K = 256: one chunk
    // hidden layers: A = h (row-major [n][256]), B(k, n') = W[n'][k]
    g.N = BP_MLP_HID; g.A = H1; g.a_m = BP_MLP_HID; g.a_k = 1; g.B = wb + o.W2; g.b_k = 1; g.b_n = BP_MLP_HID;
    g.bias = w + o.b2; g.Z = Z2; g.ldz = BP_MLP_HID; g.H = H2; g.ldh = BP_MLP_HID;
    int r = launch_gemm(EPI_BIAS_SILU, g, 1, s);
    if (r) return r;
    g.A = H2; g.B = wb + o.W3; g.bias = w + o.b3; g.Z = Z3; g.H = H3;
    r = launch_gemm(EPI_BIAS_SILU, g, 1, s);
    if (r) return r;
    g.N = BP_MLP_OUT; g.A = H3; g.B = wb + o.W4; g.bias = w + o.b4; g.F = y; g.ldf = BP_MLP_OUT; g.Z = nullptr;
    r = launch_gemm(EPI_BIAS, g, 1, s);
    prof_end(BP_PROF_MLP_FWD, s);
    return r;
}

// ------------------------------------------------------------ fused inference --
// All four layers for a block of 64 rows in one kernel; activations never leave the CU.
// Each layer is computed transposed, out^T = W h^T: the weights are the MFMA A operand and the
// activations the B operand.  A lane's accumulator holds outputs (4 (l/16) + j, l % 16) of a 16x16
// block, i.e. four consecutive features of one row, which the epilogue writes to the wavefront's
// own LDS activation rows (BF16); the next layer reads them back as B fragments of eight
// consecutive features.  The weights stream through LDS in 32-column k slices, double-buffered and
// shared by the four wavefronts.  The k order of every sum is that of bp_mlp_forward.
constexpr int kFRB = 2;                 // 16-row blocks per wavefront: each weight fragment feeds kFRB MFMAs
constexpr int kFR = 16 * kFRB;          // rows per wavefront
constexpr int kFBM = 4 * kFR;           // rows per workgroup
constexpr int kFK = 32;                 // k per slice (one 16x16x32 MFMA)
constexpr int kFKB = BP_MLP_HID / kFK;  // k slices of a hidden-layer input
constexpr int kFOB = BP_MLP_HID / 16;   // 16-feature output blocks of a hidden layer
constexpr int kFLd = kFK + 8;           // LDS row stride of a weight k slice in bf16 (32 + 8)
constexpr int kFALd = BP_MLP_HID + 8;   // LDS row stride of the activations in bf16 (256 + 8)

__device__ inline sx4 pack_bf4(float a, float b, float c, float d) {
    sx4 r;
    r[0] = (short)f2bf(a); r[1] = (short)f2bf(b); r[2] = (short)f2bf(c); r[3] = (short)f2bf(d);
    return r;
}

// One layer: acc[rb][ob] = sum_k W[16 ob + .][k] h[16 rb + row][k] over the wavefront's rows (held in act),
// for the first NOB output blocks.
template <int NOB>
__device__ inline void fused_layer(const uint16_t *__restrict__ W, const uint16_t *__restrict__ act,
                                   fx4 (&acc)[kFRB][kFOB], uint16_t *__restrict__ wsl, int t, int lane) {
#pragma unroll
    for (int rb = 0; rb < kFRB; ++rb)
#pragma unroll
        for (int ob = 0; ob < NOB; ++ob) acc[rb][ob] = fx4{0.0f, 0.0f, 0.0f, 0.0f};
    constexpr int kRows = NOB * 16;                  // weight rows (output features)
    constexpr int kBuf = BP_MLP_HID * kFLd;          // one k slice, room for 256 rows
    // thread t < kRows moves row t of a k slice: 32 bf16 = four 16-byte loads
    uint4 st0 = {}, st1 = {}, st2 = {}, st3 = {};   // (separate values: an array here is placed in LDS)
    auto fetch = [&](int kb) {
        if (t < kRows) {
            const uint4 *src = (const uint4 *)(W + (int64_t)t * BP_MLP_HID + kb * kFK);
            st0 = src[0]; st1 = src[1]; st2 = src[2]; st3 = src[3];
        }
    };
    auto put = [&](int buf) {
        if (t < kRows) {
            uint4 *dst = (uint4 *)(wsl + buf * kBuf + t * kFLd);
            dst[0] = st0; dst[1] = st1; dst[2] = st2; dst[3] = st3;
        }
    };
    fetch(0);
    put(0);
    __syncthreads();
    const uint16_t *bsrc = act + (lane & 15) * kFALd + 8 * (lane >> 4);
    for (int kb = 0; kb < kFKB; ++kb) {
        if (kb + 1 < kFKB) fetch(kb + 1);
        bf16x8 bfr[kFRB];
#pragma unroll
        for (int rb = 0; rb < kFRB; ++rb) bfr[rb] = *(const bf16x8 *)(bsrc + 16 * rb * kFALd + kFK * kb);
        const uint16_t *sl = wsl + (kb & 1) * kBuf + (lane & 15) * kFLd + 8 * (lane >> 4);
#pragma unroll
        for (int ob = 0; ob < NOB; ++ob) {
            const bf16x8 a = *(const bf16x8 *)(sl + ob * 16 * kFLd);
#pragma unroll
            for (int rb = 0; rb < kFRB; ++rb) acc[rb][ob] = mfma32(a, bfr[rb], acc[rb][ob]);
        }
        if (kb + 1 < kFKB) put((kb + 1) & 1);
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_mlp_infer(int64_t n, const float *__restrict__ w,
                                                   const uint16_t *__restrict__ wb, const float *__restrict__ x,
                                                   float *__restrict__ y, int64_t oW1, int64_t ob1, int64_t oW2,
                                                   int64_t ob2, int64_t oW3, int64_t ob3, int64_t oW4, int64_t ob4) {
    __shared__ __attribute__((aligned(16))) uint16_t wsl[2 * BP_MLP_HID * kFLd];
    __shared__ __attribute__((aligned(16))) uint16_t acts[4 * kFR * kFALd];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    uint16_t *act = acts + wv * kFR * kFALd;
    const int64_t row0 = (int64_t)blockIdx.x * kFBM + wv * kFR + (lane & 15);   // row of block rb: row0 + 16 rb
    // this lane's slot in the activation rows of block rb: row 16 rb + l%16, features 4 (l/16) + 16 kb .. + 3
    uint16_t *aslot = act + (lane & 15) * kFALd + 4 * (lane >> 4);
    // layer 1 (FP32)
    {
        const float *W1 = w + oW1, *b1 = w + ob1;
#pragma unroll
        for (int rb = 0; rb < kFRB; ++rb) {
            const int64_t row = row0 + 16 * rb;
            float x0 = 0.0f, x1 = 0.0f, x2 = 0.0f;
            if (row < n) { x0 = x[row * BP_MLP_IN]; x1 = x[row * BP_MLP_IN + 1]; x2 = x[row * BP_MLP_IN + 2]; }
            for (int kb = 0; kb < kFOB; ++kb) {
                float h[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int o = 16 * kb + 4 * (lane >> 4) + j;
                    float z = b1[o];
                    z += W1[o * BP_MLP_IN] * x0;
                    z += W1[o * BP_MLP_IN + 1] * x1;
                    z += W1[o * BP_MLP_IN + 2] * x2;
                    h[j] = silu(z);
                }
                *(sx4 *)(aslot + 16 * rb * kFALd + 16 * kb) = pack_bf4(h[0], h[1], h[2], h[3]);
            }
        }
    }
    // hidden layers 2 and 3
    fx4 acc[kFRB][kFOB];
    for (int layer = 0; layer < 2; ++layer) {
        const uint16_t *W = wb + (layer == 0 ? oW2 : oW3);
        const float *bias = w + (layer == 0 ? ob2 : ob3);
        fused_layer<kFOB>(W, act, acc, wsl, t, lane);
#pragma unroll
        for (int rb = 0; rb < kFRB; ++rb)
#pragma unroll
            for (int ob = 0; ob < kFOB; ++ob) {
                const int o = 16 * ob + 4 * (lane >> 4);
                const fx4 v = acc[rb][ob];
                *(sx4 *)(aslot + 16 * rb * kFALd + 16 * ob) =
                    pack_bf4(silu(v[0] + bias[o]), silu(v[1] + bias[o + 1]), silu(v[2] + bias[o + 2]),
                             silu(v[3] + bias[o + 3]));
            }
    }
    // output layer (144 features = 9 blocks)
    constexpr int kOB = BP_MLP_OUT / 16;
    fx4 (&out)[kFRB][kFOB] = acc;
    fused_layer<kOB>(wb + oW4, act, out, wsl, t, lane);
    const float *b4 = w + ob4;
#pragma unroll
    for (int rb = 0; rb < kFRB; ++rb) {
        const int64_t row = row0 + 16 * rb;
        if (row >= n) continue;
#pragma unroll
        for (int ob = 0; ob < kOB; ++ob) {
            const int o = 16 * ob + 4 * (lane >> 4);
            const fx4 v = out[rb][ob];
            *(float4 *)(y + row * BP_MLP_OUT + o) = float4{v[0] + b4[o], v[1] + b4[o + 1], v[2] + b4[o + 2],
                                                           v[3] + b4[o + 3]};
        }
    }
}

extern "C" int bp_mlp_infer(const float *w, const uint16_t *wb, int64_t n, const float *x, float *y, void *stream) {
    if (n < 0 || !w || !wb || !x || !y) return BP_E_ARG;
    if (n == 0) return BP_OK;
    if ((((uintptr_t)y) & 15) || (((uintptr_t)wb) & 15)) return BP_E_ARG;   // 16-byte vector access
    const int64_t blocks = (n + kFBM - 1) / kFBM;
    if (blocks > 0x7fffffffLL) return BP_E_OVERFLOW;
    hipStream_t s = (hipStream_t)stream;
    Off o = offsets();
    prof_begin(BP_PROF_MLP_FWD, s);
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)blocks), dim3(256), 0, s, n, w, wb, x, y, o.W1, o.b1, o.W2, o.b2,
                       o.W3, o.b3, o.W4, o.b4);
    prof_end(BP_PROF_MLP_FWD, s);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

// split-K factor of the weight-gradient GEMMs (K = batch): about 128 rows per slice, so that a
// 4096-row batch already gives 256 workgroups
static int wgrad_splits(int64_t n) {
    int64_t ks = (n + 127) / 128;
    return (int)(ks < 1 ? 1 : ks > 64 ? 64 : ks);
}

// The gradient as partial sums that the consumer reduces in a fixed order (GradParts): all of them
// coexist, so one kernel reduces every parameter.
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

// Gradient of parameter p from the partials, each group summed in slice / chunk order from zero.
__device__ inline float grad_of(const GradParts &P, const Off &o, int64_t p) {
    float s = 0.0f;
    if (p >= o.b4) {
        const int64_t c = p - o.b4;
        for (int y = 0; y < P.nchunk; ++y) s += P.b4[(int64_t)y * BP_MLP_OUT + c];
    } else if (p >= o.W4) {
        const int64_t i = p - o.W4, cnt = (int64_t)BP_MLP_OUT * BP_MLP_HID;
        for (int q = 0; q < P.ks; ++q) s += P.w4[q * cnt + i];
    } else if (p >= o.b3) {
        const int64_t c = p - o.b3;
        for (int y = 0; y < P.nchunk; ++y) s += P.b3[(int64_t)y * BP_MLP_HID + c];
    } else if (p >= o.W3) {
        const int64_t i = p - o.W3, cnt = (int64_t)BP_MLP_HID * BP_MLP_HID;
        for (int q = 0; q < P.ks; ++q) s += P.w3[q * cnt + i];
    } else if (p >= o.b2) {
        const int64_t c = p - o.b2;
        for (int y = 0; y < P.nchunk; ++y) s += P.b2[(int64_t)y * BP_MLP_HID + c];
    } else if (p >= o.W2) {
        const int64_t i = p - o.W2, cnt = (int64_t)BP_MLP_HID * BP_MLP_HID;
        for (int q = 0; q < P.ks; ++q) s += P.w2[q * cnt + i];
    } else if (p >= o.b1) {
        const int64_t c = p - o.b1;
        for (int y = 0; y < P.nchunk; ++y) s += P.l1[((int64_t)y * (1 + BP_MLP_NIN)) * BP_MLP_HID + c];
    } else {
        const int64_t row = p / BP_MLP_IN, k = p - row * BP_MLP_IN;   // W1[row][k]; inputs past NIN are padding
        if (k < BP_MLP_NIN)
            for (int y = 0; y < P.nchunk; ++y)
                s += P.l1[((int64_t)y * (1 + BP_MLP_NIN) + 1 + k) * BP_MLP_HID + row];
    }
    return s;
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
    return (size_t)n * BP_MLP_OUT * 2 + (size_t)n * BP_MLP_HID * (2 + 4) * 2 + part_floats(n) * 4 + 4096;
}

namespace bp {
// The backward pass up to the partials (workspace as bp_mlp_backward); *P receives their places.
int mlp_backward_parts(const float *w, const uint16_t *wb, int64_t n, const float *x, const void *act,
                       const float *dy, GradParts *P, void *ws, size_t ws_bytes, hipStream_t s) {
    if (n <= 0 || !w || !wb || !x || !act || !dy || !ws) return BP_E_ARG;
    if (ws_bytes < bp_mlp_backward_ws_bytes(n)) return BP_E_WORKSPACE;
    Off o = offsets();
    const float *Z1 = (const float *)act, *Z2 = Z1 + n * BP_MLP_HID, *Z3 = Z2 + n * BP_MLP_HID;
    const uint16_t *H1 = (const uint16_t *)(Z3 + n * BP_MLP_HID), *H2 = H1 + n * BP_MLP_HID, *H3 = H2 + n * BP_MLP_HID;
    const int ks = wgrad_splits(n);
    const int64_t kchunk = (((n + ks - 1) / ks + 31) / 32) * 32;
    Arena A(ws, ws_bytes);
    uint16_t *G4 = A.take<uint16_t>(n * BP_MLP_OUT);
    uint16_t *Gb = A.take<uint16_t>(n * BP_MLP_HID), *Gc = A.take<uint16_t>(n * BP_MLP_HID);
    float *Df = A.take<float>(n * BP_MLP_HID), *Dg = A.take<float>(n * BP_MLP_HID);
    float *part = A.take<float>((int64_t)part_floats(n));
    *P = parts_layout(part, n);
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n * BP_MLP_OUT + 255) / 256)), dim3(256), 0, s, n * BP_MLP_OUT, dy,
                       G4);
    // dW = g^T h over the batch, in ks split-K slices
    auto wgrad = [&](const uint16_t *Gt, int64_t ldg, int64_t rows, const uint16_t *Hin, const float *dst) -> int {
        GemmArgs g = {};
        g.M = rows; g.N = BP_MLP_HID; g.K = n; g.kchunk = kchunk;
        g.A = Gt; g.a_m = 1; g.a_k = ldg;          // A(m=o, k=s) = G[s][o]
        g.B = Hin; g.b_k = BP_MLP_HID; g.b_n = 1;  // B(k=s, n=i) = h[s][i]
        g.F = (float *)dst;
        return launch_gemm(EPI_PARTIAL, g, ks, s);
    };
    const int nchunk = P->nchunk;
    auto colsum = [&](const float *a, int cols, const float *dst) -> int {
        hipLaunchKernelGGL(k_colsum_part<1>, dim3((cols + 63) / 64, nchunk), dim3(256), 0, s, n, cols, a,
                           (const float *)nullptr, (float *)dst);
        return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
    };
    int r = wgrad(G4, BP_MLP_OUT, BP_MLP_OUT, H3, P->w4);
    if (r) return r;
    r = colsum(dy, BP_MLP_OUT, P->b4);
    if (r) return r;
    // dh3 = g4 W4 ; d3 = dh3 * silu'(z3)
    auto dgrad = [&](const uint16_t *Gin, int64_t kdim, const uint16_t *W, const float *Z, uint16_t *Gout,
                     float *Dout) -> int {
        GemmArgs g = {};
        g.M = n; g.N = BP_MLP_HID; g.K = kdim; g.kchunk = ((kdim + 31) / 32) * 32;
        g.A = Gin; g.a_m = kdim; g.a_k = 1;               // A(s, o) = G[s][o]
        g.B = W; g.b_k = BP_MLP_HID; g.b_n = 1;           // B(o, i) = W[o][i]
        g.Z = (float *)Z; g.ldz = BP_MLP_HID; g.H = Gout; g.ldh = BP_MLP_HID; g.F = Dout; g.ldf = BP_MLP_HID;
        return launch_gemm(EPI_DSILU, g, 1, s);
    };
    r = dgrad(G4, BP_MLP_OUT, wb + o.W4, Z3, Gb, Df);
    if (r) return r;
    r = colsum(Df, BP_MLP_HID, P->b3);
    if (r) return r;
    r = wgrad(Gb, BP_MLP_HID, BP_MLP_HID, H2, P->w3);
    if (r) return r;
    r = dgrad(Gb, BP_MLP_HID, wb + o.W3, Z2, Gc, Dg);
    if (r) return r;
    r = colsum(Dg, BP_MLP_HID, P->b2);
    if (r) return r;
    r = wgrad(Gc, BP_MLP_HID, BP_MLP_HID, H1, P->w2);
    if (r) return r;
    r = dgrad(Gc, BP_MLP_HID, wb + o.W2, Z1, Gb, Df);   // d1 in Df (fp32); its bf16 copy is unused
    if (r) return r;
    // db1 and dW1 in one pass over d1
    hipLaunchKernelGGL(k_colsum_part<1 + BP_MLP_NIN>, dim3(BP_MLP_HID / 64, nchunk), dim3(256), 0, s, n, BP_MLP_HID,
                       Df, x, (float *)P->l1);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
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
