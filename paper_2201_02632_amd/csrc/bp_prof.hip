// Optional per-kernel timing with HIP events recorded on the launch stream.
// Off by default; when on, each instrumented launch records an event pair.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "bp_internal.hpp"

namespace bp {

namespace {
struct Pair { hipEvent_t a, b; };
std::mutex g_mu;
bool g_on = false;
std::vector<Pair> g_pairs[BP_PROF_NKERNELS];
std::vector<Pair> g_free;
Pair g_open[BP_PROF_NKERNELS];
bool g_is_open[BP_PROF_NKERNELS];

bool get_pair(Pair *p) {
    if (!g_free.empty()) { *p = g_free.back(); g_free.pop_back(); return true; }
    if (hipEventCreate(&p->a) != hipSuccess) return false;
    if (hipEventCreate(&p->b) != hipSuccess) { (void)hipEventDestroy(p->a); return false; }
    return true;
}
}  // namespace

void prof_begin(int id, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on || id < 0 || id >= BP_PROF_NKERNELS) return;
    Pair p;
    if (!get_pair(&p)) return;
    if (hipEventRecord(p.a, s) != hipSuccess) { g_free.push_back(p); return; }
    g_open[id] = p;
    g_is_open[id] = true;
}

void prof_end(int id, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on || id < 0 || id >= BP_PROF_NKERNELS || !g_is_open[id]) return;
    Pair p = g_open[id];
    g_is_open[id] = false;
    if (hipEventRecord(p.b, s) != hipSuccess) { g_free.push_back(p); return; }
    g_pairs[id].push_back(p);
}

}  // namespace bp

using namespace bp;

extern "C" int bp_profiling(int enable) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (int k = 0; k < BP_PROF_NKERNELS; ++k) {
        for (auto &p : g_pairs[k]) g_free.push_back(p);
        g_pairs[k].clear();
        g_is_open[k] = false;
    }
    g_on = enable != 0;
    return BP_OK;
}

extern "C" int bp_profile_read(int kernel, double *total_ms, int64_t *launches) {
    if (kernel < 0 || kernel >= BP_PROF_NKERNELS || !total_ms || !launches) return BP_E_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    double tot = 0.0;
    for (auto &p : g_pairs[kernel]) {
        if (hipEventSynchronize(p.b) != hipSuccess) return BP_E_HIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) return BP_E_HIP;
        tot += ms;
    }
    *total_ms = tot;
    *launches = (int64_t)g_pairs[kernel].size();
    return BP_OK;
}
