// Host-side helpers shared between the libbp translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <stddef.h>
#include <stdint.h>

#include "bp_device.hpp"

extern "C" {
size_t bp_mlp_act_bytes(int64_t n);
size_t bp_mlp_backward_ws_bytes(int64_t n);
int64_t bp_mlp_nparams(void);
}

namespace bp {

const GaussRules &gauss_rules();

// bp_profile_tables on stream s; when meta_ready is given it is recorded on s after meta is written and
// before the quadratures are enqueued.
int profile_tables_launch(const bp_params *p, int64_t n, const double *sol, const int32_t *status, float *tables,
                          float *meta, hipStream_t s, hipEvent_t meta_ready);

// The second stream of the pipeline calls (solve, tables and paste in one call) and its two events, one set
// per device, created on first use with default priority.  Holders of `mu` own them for a whole call, so
// that the records and waits of two host threads never interleave.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t meta_ready = nullptr, plan_done = nullptr;
    std::mutex mu;
};
int side_stream_for_current_device(SideStream **out);
// For an error return of a call that used the second stream: `s` waits for whatever the call put there,
// so the caller may free or reuse the workspace in stream order.  Returns e (or BP_E_HIP if e is 0 and
// the join fails).
int join_side(SideStream *S, hipStream_t s, int e);

// bp_hp_paste_flat_q and bp_hp_paste_healpix_q with the set-up and plan on plan_stream (its own
// dependencies set by the caller) and the deposit on stream after plan_done and stream's own work.
int paste_flat_q_planned(const bp_params *p, int32_t npix, double pix_rad, int64_t n, const double *theta_x,
                         const double *theta_y, const double *v_los, const double *sol, const int32_t *status,
                         const float *qtables, const float *meta, float *y_map, float *b_map, float *y_comp,
                         float *b_comp, void *ws, size_t ws_bytes, size_t *ws_needed, hipStream_t stream,
                         hipStream_t plan_stream, hipEvent_t plan_done);
int paste_healpix_q_planned(const bp_params *p, int64_t nside, int64_t n, const double *theta, const double *phi,
                            const double *v_los, const double *sol, const int32_t *status, const float *qtables,
                            const float *meta, float *y_map, float *b_map, float *y_comp, float *b_comp, void *ws,
                            size_t ws_bytes, size_t *ws_needed, hipStream_t stream, hipStream_t plan_stream,
                            hipEvent_t plan_done);

// Exact surrogate q-tables (bp_surrogate_qtables_exact) for halos whose status has no bit outside ok_mask.
// Halos marked in skip (nullable) are left alone; without write_meta only the tables are written.
int qtables_exact(const bp_params *p, int64_t n, const double *sol, const int32_t *status, int32_t ok_mask,
                  float *qtables, float *meta, hipStream_t s, const uint32_t *skip = nullptr,
                  bool write_meta = true);
// The two halves of bp_surrogate_apply: the network's q-tables for the halos with a zero status and
// not marked in skip (nullable), and meta (PE0, NE0) for the halos with a zero status.
int surrogate_apply_q(int64_t n, const float *y, const float *mean, const float *std, const int32_t *status,
                      const uint32_t *skip, float *qtables, hipStream_t s);
int surrogate_apply_meta(const bp_params *p, int64_t n, const double *sol, const int32_t *status, float *meta,
                         hipStream_t s);

// The surrogate network's gradient as partial sums that their consumer reduces in a fixed order:
// split-K slices of the weight-gradient products (W4, W3, W2) and row-chunk column sums (b4, b3, b2,
// and the first layer's bias and input columns).
struct GradParts {
    const float *w4, *w3, *w2;   // [ks][rows * 256]
    const float *b4, *b3, *b2;   // [nchunk][cols]
    const float *l1;             // [nchunk][1 + BP_MLP_NIN][256]
    int ks, nchunk;
};
// bp_mlp_backward up to the partials (same arguments and workspace), and one Adam step from them
// (bp_mlp_adam's update with the gradient reduced on the fly; the gradient is also written to g).
int mlp_backward_parts(const float *w, const uint16_t *wb, int64_t n, const float *x, const void *act,
                       const float *dy, GradParts *P, void *ws, size_t ws_bytes, hipStream_t s);
// The places in a backward workspace (bp_mlp_backward_ws_bytes(n) bytes) of the BF16 output
// gradient [n][BP_MLP_OUT] and of the partials; the b4 partials are the producer's of that gradient.
int mlp_backward_layout(void *ws, size_t ws_bytes, int64_t n, uint16_t **g4, GradParts *P);
// The backward from the BF16 output gradient and the b4 partials already in the workspace.
int mlp_backward_g4(const uint16_t *wb, int64_t n, const float *x, const void *act, void *ws, size_t ws_bytes,
                    hipStream_t s);
// The forward pass of a training batch drawn by train_row from xdata [ndata][BP_MLP_IN]; the drawn
// inputs (the first BP_MLP_NIN of each row) are also written to xb [n][BP_MLP_IN] for the backward.
int mlp_forward_train(const float *w, const uint16_t *wb, int64_t n, int64_t ndata, uint64_t seed, int64_t step,
                      const float *xdata, float *xb, void *act, float *y, hipStream_t s);

// SplitMix64 (Steele, Lea & Flood 2014), a counter-based generator: row i of the training batch of
// step `step` is data row (splitmix64(seed ^ splitmix64(step * 0x100000001B3 + i)) >> 11) mod ndata.
__device__ inline uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
__device__ inline int64_t train_row(uint64_t seed, int64_t step, int64_t i, int64_t ndata) {
    const uint64_t h = splitmix64(seed ^ splitmix64((uint64_t)step * 0x100000001B3ull + (uint64_t)i));
    return (int64_t)((h >> 11) % (uint64_t)ndata);
}

// round-to-nearest-even FP32 -> BF16 (gfx950 converts in hardware, v_cvt_pk_bf16_f32)
__device__ inline uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
int mlp_adam_parts(const GradParts &P, float *w, float *m, float *v, float *g, uint16_t *wb, float lr, float b1,
                   float b2, float eps, int64_t step, hipStream_t s);

// Validate the model parameters (every entry point that takes bp_params): BP_OK or BP_E_ARG.
// Gamma must be the paper's 1.2, the polytropic index the kernels are written for.
int check_params(const bp_params *p);

// Bump allocator over a caller-provided workspace; sizes rounded to 256 B.
struct Arena {
    char *base;
    size_t cap, used;
    explicit Arena(void *p, size_t c) : base((char *)p), cap(c), used(0) {}
    template <class T>
    T *take(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
        T *r = (T *)(base ? base + used : nullptr);
        used += bytes;
        return r;
    }
    bool fits() const { return used <= cap && base != nullptr; }
};

// Exclusive prefix sum of n uint32 values (in != out allowed or equal).
size_t scan_ws_bytes(int64_t n);
int scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, void *ws, hipStream_t s);

// Stable LSD radix sort of (key, value) uint32 pairs on key bits [0, bits).
// Ping-pongs between (k0, v0) and (k1, v1); returns via *result_in_k1
// whether the sorted data ended in k1/v1.
size_t radix_ws_bytes(int64_t n);
int radix_sort_u32(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n, int bits, void *ws,
                   hipStream_t s, bool *result_in_k1);
int radix_sort_u64(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n, int bits, void *ws,
                   hipStream_t s, bool *result_in_k1);

// Optional kernel timing (bp_profiling): event pair around one launch.
void prof_begin(int id, hipStream_t s);
void prof_end(int id, hipStream_t s);

// chi(z) and tau(z) on the uniform grid of bp_cosmo.hpp (kNZ doubles each).
int cosmo_tables(const bp_params &P, double *chi_t, double *tau_t, hipStream_t s);

// Fill n uint32 with a value (a kernel, safe under graph capture).
int fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);

}  // namespace bp
