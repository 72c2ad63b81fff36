// Surrogate lifecycle behind one caller-owned device state buffer: initialisation, training from
// exact solves, save / load as a flat blob, and the HP pastes that route every halo on the device
// (network-seeded solve inside the training domain, the exact scan solve outside it or where the
// seeded root search fails) into one q-table deposit.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include "bp_device.hpp"
#include "bp_internal.hpp"

namespace bp {

// State layout: each array starts on a 256-byte boundary.
struct SurLayout {
    size_t off[BP_SUR_NARRAYS];
    size_t total;
};
static SurLayout sur_layout() {
    const int64_t np = bp_mlp_nparams();
    const size_t bytes[BP_SUR_NARRAYS] = {(size_t)np * 4, (size_t)np * 2, (size_t)np * 4, (size_t)np * 4,
                                          (size_t)np * 4, (size_t)BP_MLP_OUT * 4, (size_t)BP_MLP_OUT * 4};
    SurLayout L;
    size_t o = 0;
    for (int a = 0; a < BP_SUR_NARRAYS; ++a) {
        L.off[a] = o;
        o += (bytes[a] + 255) & ~(size_t)255;
    }
    L.total = o;
    return L;
}

// counter-based normal deviates: SplitMix64 of (seed, index) -> two uniforms -> Box-Muller
__device__ inline uint64_t smix(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// He initialisation: W_l ~ N(0, 2 / fan_in) (fan_in 3, 256, 256, 256), biases 0, the padding columns of
// W1 (inputs 3..15) 0; Adam moments and gradient 0; output mean 0 and standard deviation 1.
__global__ void k_sur_init(uint64_t seed, int64_t np, float *__restrict__ w, float *__restrict__ m,
                           float *__restrict__ v, float *__restrict__ g, float *__restrict__ mean,
                           float *__restrict__ sd) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < BP_MLP_OUT) { mean[e] = 0.0f; sd[e] = 1.0f; }
    if (e >= np) return;
    const int64_t H = BP_MLP_HID, I = BP_MLP_IN;
    const int64_t oW1 = 0, ob1 = H * I, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H, ob3 = oW3 + H * H,
                  oW4 = ob3 + H, ob4 = oW4 + (int64_t)BP_MLP_OUT * H;
    double sdev = 0.0;
    if (e < ob1) sdev = (e % I) < BP_MLP_NIN ? sqrt(2.0 / BP_MLP_NIN) : 0.0;
    else if ((e >= oW2 && e < ob2) || (e >= oW3 && e < ob3) || (e >= oW4 && e < ob4)) sdev = sqrt(2.0 / H);
    float val = 0.0f;
    if (sdev > 0.0) {
        const uint64_t h1 = smix(seed ^ smix(2 * (uint64_t)e)), h2 = smix(seed ^ smix(2 * (uint64_t)e + 1));
        const double u1 = ((double)(h1 >> 11) + 1.0) * 0x1.0p-53, u2 = (double)(h2 >> 11) * 0x1.0p-53;
        val = (float)(sdev * sqrt(-2.0 * log(u1)) * cos(2.0 * kPi * u2));
    }
    w[e] = val; m[e] = 0.0f; v[e] = 0.0f; g[e] = 0.0f;
}

// halos the seeded solve leaves to the exact scan: outside the training domain, no root near the
// estimate, or a non-finite trial (invalid inputs and stars above the baryon mass stay as they are)
constexpr int32_t kRouteBits = BP_S_OUT_OF_DOMAIN | BP_S_NO_BRACKET | BP_S_NONFINITE;

__global__ void k_route_flags(int64_t n, const int32_t *__restrict__ st, uint32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    flag[i] = (i < n && (st[i] & kRouteBits)) ? 1u : 0u;
}

__global__ void k_route_gather(int64_t n, const uint32_t *__restrict__ flag, const uint32_t *__restrict__ off,
                               const double *__restrict__ M, const double *__restrict__ c,
                               const double *__restrict__ z, int64_t *__restrict__ idx, double *__restrict__ Ms,
                               double *__restrict__ cs, double *__restrict__ zs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    const uint32_t j = off[i];
    idx[j] = i; Ms[j] = M[i]; cs[j] = c[i]; zs[j] = z[i];
}

// the scanned halos' solution, status, q-table row and meta back into the full arrays; a halo with
// several roots keeps the first (as the exact path does) and is pasted like any solved halo
__global__ void k_route_scatter(int64_t n, int64_t m, const int64_t *__restrict__ idx,
                                const double *__restrict__ sol_s, const int32_t *__restrict__ st_s,
                                const float *__restrict__ qt_s, const float *__restrict__ meta_s,
                                double *__restrict__ sol, int32_t *__restrict__ st, float *__restrict__ qt,
                                float *__restrict__ meta) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * 2 * BP_MLP_NQ) return;
    const int64_t j = e / (2 * BP_MLP_NQ);
    const int k = (int)(e - j * 2 * BP_MLP_NQ);
    const int64_t i = idx[j];
    const int32_t s = st_s[j] & ~BP_S_MULTI_ROOT;
    qt[i * 2 * BP_MLP_NQ + k] = qt_s[j * 2 * BP_MLP_NQ + k];
    if (k < BP_SOL_NFIELDS) sol[(int64_t)k * n + i] = sol_s[(int64_t)k * m + j];
    else if (k < BP_SOL_NFIELDS + BP_META_NFIELDS) {
        const int f = k - BP_SOL_NFIELDS;
        meta[(int64_t)f * n + i] = meta_s[(int64_t)f * m + j];
    } else if (k == BP_SOL_NFIELDS + BP_META_NFIELDS) st[i] = s;
}
static_assert(BP_SOL_NFIELDS + BP_META_NFIELDS < 2 * BP_MLP_NQ, "one thread per copied field");

struct SurViews {
    float *w, *m, *v, *g, *mean, *sd;
    uint16_t *wb;
};
static SurViews views(void *state) {
    const SurLayout L = sur_layout();
    char *b = (char *)state;
    SurViews V;
    V.w = (float *)(b + L.off[BP_SUR_W]); V.wb = (uint16_t *)(b + L.off[BP_SUR_WBF16]);
    V.m = (float *)(b + L.off[BP_SUR_M]); V.v = (float *)(b + L.off[BP_SUR_V]); V.g = (float *)(b + L.off[BP_SUR_G]);
    V.mean = (float *)(b + L.off[BP_SUR_MEAN]); V.sd = (float *)(b + L.off[BP_SUR_STD]);
    return V;
}

// Everything up to the deposit: network, seeded solve, tables, the routed halos' exact solve and
// tables.  Returns BP_OK with the arrays filled, or BP_E_WORKSPACE with *need set.
//
// The solution, status and meta of every halo are final before the q-tables of the halos solved by
// the seeded solve are enqueued (the routed halos' own q-tables come with their exact solve), so the
// paste's plan may run on a second stream hs beside those q-tables: `routed` is recorded on s at that
// point and hs waits for it.  The q-table kernels skip the routed halos by their flag (their status is
// zero again after the scatter); the caller orders the deposit after both streams.
struct Routed {
    double *sol;
    int32_t *st;
    float *qt, *meta;
    int64_t nfall;
    size_t used;
};
static int route_halos(const bp_params *p, const void *state, int32_t tables, int64_t n, const double *M,
                       const double *c, const double *z, void *ws, size_t ws_bytes, size_t *need, hipStream_t s,
                       hipStream_t hs, hipEvent_t routed, Routed *R) {
    SurViews V = views((void *)state);
    Arena A(ws, ws_bytes);
    float *x = A.take<float>(n * BP_MLP_IN), *y = A.take<float>(n * BP_MLP_OUT);
    double *sol = A.take<double>(n * BP_SOL_NFIELDS);
    int32_t *st = A.take<int32_t>(n);
    float *qt = A.take<float>(n * 2 * BP_MLP_NQ), *meta = A.take<float>(n * BP_META_NFIELDS);
    uint32_t *flag = A.take<uint32_t>(n + 1), *off = A.take<uint32_t>(n + 1);
    char *scan_ws = A.take<char>(scan_ws_bytes(n + 1));
    if (!A.fits()) { *need = A.used + 4096; return BP_E_WORKSPACE; }
    int e;
    if ((e = bp_surrogate_features(n, M, c, z, x, s))) return e;
    if ((e = bp_mlp_infer(V.w, V.wb, n, x, y, s))) return e;
    if ((e = bp_surrogate_solve(p, n, M, c, z, y, V.mean, V.sd, sol, st, s))) return e;
    if ((e = surrogate_apply_meta(p, n, sol, st, meta, s))) return e;
    const unsigned nb = (unsigned)((n + 256) / 256);
    hipLaunchKernelGGL(k_route_flags, dim3(nb), dim3(256), 0, s, n, st, flag);
    if ((e = scan_exclusive_u32(flag, off, n + 1, scan_ws, s))) return e;
    uint32_t m32 = 0;
    if (hipMemcpyAsync(&m32, off + n, sizeof(m32), hipMemcpyDeviceToHost, s) != hipSuccess) return BP_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return BP_E_HIP;
    const int64_t m = m32;
    R->sol = sol; R->st = st; R->qt = qt; R->meta = meta; R->nfall = m;
    int64_t *idx = nullptr;
    double *Ms = nullptr, *cs = nullptr, *zs = nullptr, *sol_s = nullptr;
    int32_t *st_s = nullptr;
    float *qt_s = nullptr, *meta_s = nullptr;
    if (m > 0) {
        idx = A.take<int64_t>(m);
        Ms = A.take<double>(m); cs = A.take<double>(m); zs = A.take<double>(m);
        sol_s = A.take<double>(m * BP_SOL_NFIELDS);
        st_s = A.take<int32_t>(m);
        qt_s = A.take<float>(m * 2 * BP_MLP_NQ); meta_s = A.take<float>(m * BP_META_NFIELDS);
        if (!A.fits()) { *need = A.used + 4096; return BP_E_WORKSPACE; }
    }
    R->used = A.used;
    if (m > 0) {
        hipLaunchKernelGGL(k_route_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, flag, off, M, c, z,
                           idx, Ms, cs, zs);
        if ((e = bp_icm_solve(p, m, Ms, cs, zs, sol_s, st_s, s))) return e;
        // a halo with several roots is pasted with the first; the q-table kernel skips non-zero status
        if ((e = qtables_exact(p, m, sol_s, st_s, BP_S_MULTI_ROOT, qt_s, meta_s, s))) return e;
        hipLaunchKernelGGL(k_route_scatter, dim3((unsigned)((m * 2 * BP_MLP_NQ + 255) / 256)), dim3(256), 0, s, n,
                           m, idx, sol_s, st_s, qt_s, meta_s, sol, st, qt, meta);
        if (hipGetLastError() != hipSuccess) return BP_E_HIP;
    }
    // solution, status and meta are final: the paste's plan may start on hs while the q-tables of the
    // other halos run on s
    if (hs != s && (hipEventRecord(routed, s) != hipSuccess || hipStreamWaitEvent(hs, routed, 0) != hipSuccess))
        return BP_E_HIP;
    if (tables == BP_SUR_TABLES_EXACT) e = qtables_exact(p, n, sol, st, 0, qt, meta, s, flag, false);
    else e = surrogate_apply_q(n, y, V.mean, V.sd, st, flag, qt, s);
    if (e) return e;
    return BP_OK;
}

}  // namespace bp

using namespace bp;

extern "C" size_t bp_surrogate_state_bytes(void) { return sur_layout().total; }

// the state buffer: non-null and 256-byte aligned (its arrays are then 16-byte aligned for the
// kernels' vector accesses)
static bool state_ok(const void *state) { return state && !((uintptr_t)state & 255); }

extern "C" size_t bp_surrogate_state_offset(int32_t array) {
    if (array < 0 || array >= BP_SUR_NARRAYS) return (size_t)-1;
    return sur_layout().off[array];
}

extern "C" int bp_surrogate_init(void *state, uint64_t seed, void *stream) {
    if (!state_ok(state)) return BP_E_ARG;
    SurViews V = views(state);
    const int64_t np = bp_mlp_nparams();
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_sur_init, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, seed, np, V.w, V.m, V.v, V.g,
                       V.mean, V.sd);
    if (hipGetLastError() != hipSuccess) return BP_E_HIP;
    return bp_mlp_to_bf16(np, V.w, V.wb, stream);
}

// blob: 64-byte header (magic, format, parameter count, output width, Adam step) then the FP32
// arrays w, m, v, mean, std in that order
namespace {
constexpr uint64_t kBlobMagic = 0x31766c6f62707362ull;   // "bpsblov1"
struct BlobHead { uint64_t magic, format, nparams, nout, step, pad[3]; };
size_t blob_bytes() {
    const int64_t np = bp_mlp_nparams();
    return sizeof(BlobHead) + (size_t)(3 * np + 2 * BP_MLP_OUT) * 4;
}
}  // namespace

extern "C" size_t bp_surrogate_blob_bytes(void) { return blob_bytes(); }

extern "C" int bp_surrogate_save(const void *state, int64_t step, void *blob, size_t blob_bytes_, void *stream) {
    if (!state_ok(state) || !blob || blob_bytes_ < blob_bytes() || step < 0) return BP_E_ARG;
    SurViews V = views((void *)state);
    const int64_t np = bp_mlp_nparams();
    BlobHead H = {kBlobMagic, 1, (uint64_t)np, BP_MLP_OUT, (uint64_t)step, {0, 0, 0}};
    memcpy(blob, &H, sizeof(H));
    char *b = (char *)blob + sizeof(H);
    hipStream_t s = (hipStream_t)stream;
    const void *src[5] = {V.w, V.m, V.v, V.mean, V.sd};
    const size_t len[5] = {(size_t)np * 4, (size_t)np * 4, (size_t)np * 4, BP_MLP_OUT * 4, BP_MLP_OUT * 4};
    for (int a = 0; a < 5; ++a) {
        if (hipMemcpyAsync(b, src[a], len[a], hipMemcpyDeviceToHost, s) != hipSuccess) return BP_E_HIP;
        b += len[a];
    }
    return hipStreamSynchronize(s) == hipSuccess ? BP_OK : BP_E_HIP;
}

extern "C" int bp_surrogate_load(void *state, const void *blob, size_t blob_bytes_, int64_t *step, void *stream) {
    if (!state_ok(state) || !blob || blob_bytes_ < sizeof(BlobHead)) return BP_E_ARG;
    BlobHead H;
    memcpy(&H, blob, sizeof(H));
    const int64_t np = bp_mlp_nparams();
    if (H.magic != kBlobMagic || H.format != 1 || H.nparams != (uint64_t)np || H.nout != BP_MLP_OUT ||
        blob_bytes_ < blob_bytes())
        return BP_E_ARG;
    SurViews V = views(state);
    const char *b = (const char *)blob + sizeof(H);
    hipStream_t s = (hipStream_t)stream;
    void *dst[5] = {V.w, V.m, V.v, V.mean, V.sd};
    const size_t len[5] = {(size_t)np * 4, (size_t)np * 4, (size_t)np * 4, BP_MLP_OUT * 4, BP_MLP_OUT * 4};
    for (int a = 0; a < 5; ++a) {
        if (hipMemcpyAsync(dst[a], b, len[a], hipMemcpyHostToDevice, s) != hipSuccess) return BP_E_HIP;
        b += len[a];
    }
    int e = bp_mlp_to_bf16(np, V.w, V.wb, stream);
    if (e) return e;
    if (hipStreamSynchronize(s) != hipSuccess) return BP_E_HIP;   // the host blob may go away after return
    if (step) *step = (int64_t)H.step;
    return BP_OK;
}

extern "C" int bp_surrogate_fit(const bp_params *p, void *state, int64_t n, const double *M, const double *c,
                                const double *z, int64_t steps, int64_t batch, float lr0, float lr1, uint64_t seed,
                                int64_t step0, void *ws, size_t ws_bytes, size_t *ws_needed, void *stream) {
    if (check_params(p) || !state_ok(state) || n <= 0 || !M || !c || !z || steps < 0 || batch <= 0 || step0 < 0 || !ws_needed)
        return BP_E_ARG;
    if (n > ((int64_t)1 << 31)) return BP_E_OVERFLOW;
    SurViews V = views(state);
    Arena A(ws, ws_bytes);
    double *sol = A.take<double>(n * BP_SOL_NFIELDS);
    int32_t *st = A.take<int32_t>(n);
    float *tab = A.take<float>(n * BP_TAB_STRIDE), *meta = A.take<float>(n * BP_META_NFIELDS);
    float *x = A.take<float>(n * BP_MLP_IN), *t = A.take<float>(n * BP_MLP_OUT);
    const size_t tws = bp_surrogate_train_ws_bytes(batch);
    char *train_ws = A.take<char>(tws);
    *ws_needed = A.used + 4096;
    if (!A.fits()) return BP_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    int e;
    if ((e = bp_icm_solve(p, n, M, c, z, sol, st, s))) return e;
    if ((e = bp_profile_tables(p, n, sol, st, tab, meta, s))) return e;
    if ((e = bp_surrogate_targets(p, n, sol, st, tab, meta, t, s))) return e;
    if ((e = bp_surrogate_features(n, M, c, z, x, s))) return e;
    if ((e = bp_surrogate_stats(n, t, V.mean, V.sd, s))) return e;
    return bp_surrogate_train(V.w, V.wb, V.m, V.v, V.g, V.mean, V.sd, n, x, t, steps, batch, lr0, lr1, seed, step0,
                              nullptr, train_ws, tws, stream);
}

extern "C" int bp_surrogate_paste_flat(const bp_params *p, const void *state, int32_t tables, int32_t npix,
                                       double pix_rad, int64_t n, const double *M, const double *c, const double *z,
                                       const double *theta_x, const double *theta_y, const double *v_los,
                                       float *y_map, float *b_map, float *y_comp, float *b_comp, void *ws,
                                       size_t ws_bytes, size_t *ws_needed, int64_t *n_fallback, void *stream) {
    if (check_params(p) || !state_ok(state) || (tables != BP_SUR_TABLES_EXACT && tables != BP_SUR_TABLES_NETWORK) || npix <= 0 ||
        npix > 65536 || !(pix_rad > 0) || n < 0 || !ws_needed || !y_map || !b_map)
        return BP_E_ARG;
    if (n > 0 && (!M || !c || !z || !theta_x || !theta_y || !v_los)) return BP_E_ARG;
    if (n >= 0x7fffffffLL) return BP_E_OVERFLOW;
    if (n_fallback) *n_fallback = 0;
    if (n == 0) { *ws_needed = 0; return BP_OK; }
    hipStream_t s = (hipStream_t)stream;
    SideStream *S = nullptr;
    int e = side_stream_for_current_device(&S);
    if (e) return e;
    std::lock_guard<std::mutex> lock(S->mu);
    Routed R;
    size_t need = 0;
    e = route_halos(p, state, tables, n, M, c, z, ws, ws_bytes, &need, s, S->s, S->meta_ready, &R);
    if (e == BP_E_WORKSPACE) *ws_needed = need;
    if (e) return join_side(S, s, e);
    size_t dneed = 0;
    e = paste_flat_q_planned(p, npix, pix_rad, n, theta_x, theta_y, v_los, R.sol, R.st, R.qt, R.meta, y_map, b_map,
                             y_comp, b_comp, (char *)ws + R.used, ws_bytes - R.used, &dneed, s, S->s, S->plan_done);
    *ws_needed = R.used + dneed;
    if (e) return join_side(S, s, e);
    if (n_fallback) *n_fallback = R.nfall;
    return BP_OK;
}

extern "C" int bp_surrogate_paste_healpix(const bp_params *p, const void *state, int32_t tables, int64_t nside,
                                          int64_t n, const double *M, const double *c, const double *z,
                                          const double *theta, const double *phi, const double *v_los, float *y_map,
                                          float *b_map, float *y_comp, float *b_comp, void *ws, size_t ws_bytes,
                                          size_t *ws_needed, int64_t *n_fallback, void *stream) {
    if (check_params(p) || !state_ok(state) || (tables != BP_SUR_TABLES_EXACT && tables != BP_SUR_TABLES_NETWORK) || nside < 1 ||
        nside > 8192 || n < 0 || !ws_needed || !y_map || !b_map)
        return BP_E_ARG;
    if (n > 0 && (!M || !c || !z || !theta || !phi || !v_los)) return BP_E_ARG;
    if (n >= 0x7fffffffLL) return BP_E_OVERFLOW;
    if (n_fallback) *n_fallback = 0;
    if (n == 0) { *ws_needed = 0; return BP_OK; }
    hipStream_t s = (hipStream_t)stream;
    SideStream *S = nullptr;
    int e = side_stream_for_current_device(&S);
    if (e) return e;
    std::lock_guard<std::mutex> lock(S->mu);
    Routed R;
    size_t need = 0;
    e = route_halos(p, state, tables, n, M, c, z, ws, ws_bytes, &need, s, S->s, S->meta_ready, &R);
    if (e == BP_E_WORKSPACE) *ws_needed = need;
    if (e) return join_side(S, s, e);
    size_t dneed = 0;
    e = paste_healpix_q_planned(p, nside, n, theta, phi, v_los, R.sol, R.st, R.qt, R.meta, y_map, b_map, y_comp,
                                b_comp, (char *)ws + R.used, ws_bytes - R.used, &dneed, s, S->s, S->plan_done);
    *ws_needed = R.used + dneed;
    if (e) return join_side(S, s, e);
    if (n_fallback) *n_fallback = R.nfall;
    return BP_OK;
}
