// Launch timing with HIP events for the measurement entry points
// (kgev_profile_begin / kgev_profile_end).
#include <vector>

#include "kernels.hpp"

namespace kgev {

struct Profiler {
    int phase = PH_NONE;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    int64_t launches = 0;
    double bytes = 0, flops = 0;
};

thread_local Profiler* g_prof = nullptr;

static hipEvent_t next_event(Profiler* p)
{
    if (p->used == p->pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        p->pool.push_back(e);
    }
    return p->pool[p->used++];
}

// Launches captured into a graph are not timed: the runtime does not time
// events recorded by graph nodes.
static bool capturing(hipStream_t st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

void prof_before(int phase, hipStream_t st)
{
    Profiler* p = g_prof;
    if (!p || p->phase != phase || capturing(st)) return;
    hipEvent_t e = next_event(p);
    if (e) (void)hipEventRecord(e, st);
}

void prof_after(int phase, hipStream_t st, double bytes, double flops)
{
    Profiler* p = g_prof;
    if (!p || p->phase != phase || capturing(st)) return;
    hipEvent_t e = next_event(p);
    if (e) (void)hipEventRecord(e, st);
    p->launches += 1;
    p->bytes += bytes;
    p->flops += flops;
}

Profiler* prof_start(int phase, size_t reserve)
{
    Profiler* p = new Profiler;
    p->phase = phase;
    p->pool.reserve(reserve);
    for (size_t q = 0; q < reserve; ++q) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) break;
        p->pool.push_back(e);
    }
    g_prof = p;
    return p;
}

bool prof_stop(Profiler* p, int64_t* launches, double* ms, double* bytes, double* flops)
{
    if (g_prof == p) g_prof = nullptr;
    double total = 0;
    bool ok = true;
    for (size_t q = 0; q + 1 < p->used; q += 2) {
        if (hipEventSynchronize(p->pool[q + 1]) != hipSuccess) { ok = false; break; }
        float t = 0;
        if (hipEventElapsedTime(&t, p->pool[q], p->pool[q + 1]) != hipSuccess) { ok = false; break; }
        total += t;
    }
    if (launches) *launches = p->launches;
    if (ms) *ms = total;
    if (bytes) *bytes = p->bytes;
    if (flops) *flops = p->flops;
    for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
    delete p;
    return ok;
}

}  // namespace kgev
