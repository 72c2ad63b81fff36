// Prefix sums and a stable LSD radix sort for the (tile, halo) pair lists.
//
// Both run in fixed-size chunks of 4096 items per 256-lane workgroup.  The
// radix scatter ranks equal digits inside a wavefront with 8 ballots (one per
// digit bit), so the order of equal keys is the input order: the sort is
// stable and therefore deterministic.
#include <hip/hip_runtime.h>

#include "bp_internal.hpp"

namespace bp {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kChunk = kScanThreads * kScanItems;  // 4096

// Block-wide exclusive scan of one value per thread (256 threads, 4 waves).
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *total, uint32_t *lds /* >= 4 */) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[w] = x;
    __syncthreads();
    uint32_t wp = 0, tot = 0;
    for (int q = 0; q < 4; ++q) { uint32_t c = lds[q]; if (q < w) wp += c; tot += c; }
    __syncthreads();
    *total = tot;
    return wp + x - v;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const uint32_t *__restrict__ in, uint32_t *__restrict__ bsum,
                                                              int64_t n) {
    __shared__ uint32_t lds[4];
    int64_t base = (int64_t)blockIdx.x * kChunk;
    uint32_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint32_t tot;
    block_exclusive_scan(s, &tot, lds);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Exclusive scan of each chunk, offset by boff[block] (nullptr = 0).
__global__ void __launch_bounds__(kScanThreads) k_scan_down(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                            const uint32_t *__restrict__ boff, int64_t n) {
    __shared__ uint32_t lds[4];
    int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems], s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        v[k] = (i < n) ? in[i] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t pre = block_exclusive_scan(s, &tot, lds) + (boff ? boff[blockIdx.x] : 0u);
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = pre;
        pre += v[k];
    }
}

size_t scan_ws_bytes(int64_t n) {
    size_t total = 0;
    while (n > kChunk) {
        int64_t nb = (n + kChunk - 1) / kChunk;
        total += 2 * (((size_t)nb * 4 + 255) & ~(size_t)255);
        n = nb;
    }
    return total + 256;
}

int scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, void *ws, hipStream_t s) {
    if (n <= 0) return BP_OK;
    if (n <= kChunk) {
        hipLaunchKernelGGL(k_scan_down, dim3(1), dim3(kScanThreads), 0, s, in, out, (const uint32_t *)nullptr, n);
        return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
    }
    int64_t nb = (n + kChunk - 1) / kChunk;
    Arena A(ws, SIZE_MAX);
    uint32_t *bsum = A.take<uint32_t>(nb);
    uint32_t *boff = A.take<uint32_t>(nb);
    char *rest = (char *)ws + A.used;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, bsum, n);
    int e = scan_exclusive_u32(bsum, boff, nb, rest, s);
    if (e) return e;
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, boff, n);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

// ---------------------------------------------------------------- radix --
template <class K>
__global__ void __launch_bounds__(256) k_radix_hist(const K *__restrict__ keys, uint32_t *__restrict__ hist,
                                                    int64_t n, int shift, int nb) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kChunk;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)k * 256 + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// One chunk per workgroup: the chunk is first ranked into LDS in digit order (stable: rounds in input
// order, waves in order inside a round, ballot ranks inside a wave), then written out by consecutive
// lanes, so each digit's run of the chunk (16 items on average) leaves as contiguous stores instead of
// 256 scattered 4-byte stores per round, each in a different cache line.
template <class K>
__global__ void __launch_bounds__(256) k_radix_scatter(const K *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                       K *__restrict__ kout, uint32_t *__restrict__ vout,
                                                       const uint32_t *__restrict__ hist,
                                                       const uint32_t *__restrict__ offs, int64_t n, int shift, int nb) {
    __shared__ K skey[kChunk];
    __shared__ uint32_t sval[kChunk];
    __shared__ uint32_t gbase[256];   // first output slot of each digit for this chunk
    __shared__ uint32_t lbase[256];   // first LDS slot of each digit (the chunk's own digit prefix)
    __shared__ uint32_t run[256];     // items of each digit placed so far
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint32_t lds[4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    gbase[t] = offs[(int64_t)t * nb + blockIdx.x];
    uint32_t tot;
    lbase[t] = block_exclusive_scan(hist[(int64_t)t * nb + blockIdx.x], &tot, lds);
    run[t] = 0;
    const int64_t start = (int64_t)blockIdx.x * kChunk;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int round = 0; round < kScanItems; ++round) {
        wcnt[0][t] = 0; wcnt[1][t] = 0; wcnt[2][t] = 0; wcnt[3][t] = 0;
        __syncthreads();
        int64_t idx = start + (int64_t)round * 256 + t;
        bool valid = idx < n;
        K key = valid ? kin[idx] : (K)0;
        uint32_t val = valid ? vin[idx] : 0u;
        uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t mask = __ballot(valid);
        for (int bit = 0; bit < 8; ++bit) {
            uint64_t bb = __ballot((d >> bit) & 1u);
            mask &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        uint32_t rank = (uint32_t)__popcll(mask & below);
        if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(mask);
        __syncthreads();
        if (valid) {
            uint32_t pre = 0;
            for (int q = 0; q < w; ++q) pre += wcnt[q][d];
            const uint32_t pos = lbase[d] + run[d] + pre + rank;
            skey[pos] = key;
            sval[pos] = val;
        }
        __syncthreads();
        run[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
    }
    __syncthreads();
    // tot = the chunk's item count (its digit counts summed)
    for (uint32_t j = t; j < tot; j += 256) {
        const K key = skey[j];
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        const uint32_t pos = gbase[d] + (j - lbase[d]);
        kout[pos] = key;
        vout[pos] = sval[j];
    }
}

size_t radix_ws_bytes(int64_t n) {
    int64_t nb = (n + kChunk - 1) / kChunk;
    size_t hist = (((size_t)nb * 256 * 4) + 255) & ~(size_t)255;
    return 2 * hist + scan_ws_bytes(nb * 256) + 256;
}

template <class K>
static int radix_sort_impl(K *k0, uint32_t *v0, K *k1, uint32_t *v1, int64_t n, int bits, void *ws, hipStream_t s,
                           bool *result_in_k1) {
    *result_in_k1 = false;
    if (n <= 1 || bits <= 0) return BP_OK;
    int64_t nb = (n + kChunk - 1) / kChunk;
    if (nb * 256 > 0x7fffffffLL) return BP_E_OVERFLOW;
    Arena A(ws, SIZE_MAX);
    uint32_t *hist = A.take<uint32_t>(nb * 256);
    uint32_t *offs = A.take<uint32_t>(nb * 256);
    void *sws = (char *)ws + A.used;
    K *ki = k0, *ko = k1;
    uint32_t *vi = v0, *vo = v1;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist<K>, dim3((unsigned)nb), dim3(256), 0, s, ki, hist, n, shift, (int)nb);
        int e = scan_exclusive_u32(hist, offs, nb * 256, sws, s);
        if (e) return e;
        hipLaunchKernelGGL(k_radix_scatter<K>, dim3((unsigned)nb), dim3(256), 0, s, ki, vi, ko, vo, hist, offs, n,
                           shift, (int)nb);
        if (hipGetLastError() != hipSuccess) return BP_E_HIP;
        K *tk = ki; ki = ko; ko = tk;
        uint32_t *tv = vi; vi = vo; vo = tv;
        *result_in_k1 = !*result_in_k1;
    }
    return BP_OK;
}

int radix_sort_u32(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n, int bits, void *ws,
                   hipStream_t s, bool *result_in_k1) {
    return radix_sort_impl<uint32_t>(k0, v0, k1, v1, n, bits, ws, s, result_in_k1);
}

int radix_sort_u64(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n, int bits, void *ws,
                   hipStream_t s, bool *result_in_k1) {
    return radix_sort_impl<uint64_t>(k0, v0, k1, v1, n, bits, ws, s, result_in_k1);
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

int fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return BP_OK;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff) return BP_E_OVERFLOW;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError() == hipSuccess ? BP_OK : BP_E_HIP;
}

}  // namespace bp
