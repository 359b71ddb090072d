// Launch timing with HIP events for the measurement entry points
// (kgev_profile_begin / kgev_profile_end).
#include <vector>

#include "kernels.hpp"

namespace kgev {

// Every stride-th launch of the phase is timed by events carried in its own
// dispatch (timing every launch of a phase with thousands of short launches
// would slow what is measured).
struct Profiler {
    int phase = PH_NONE;
    int stride = 1;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    int64_t seen = 0;          // launches of the phase
    int64_t launches = 0;      // timed launches
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

ProfLaunch prof_launch_begin(int phase, hipStream_t st)
{
    ProfLaunch pl;
    Profiler* p = g_prof;
    if (!p || p->phase != phase || capturing(st)) return pl;
    if (p->seen % p->stride != 0) return pl;
    const size_t mark = p->used;
    pl.start = next_event(p);
    pl.stop = pl.start ? next_event(p) : nullptr;
    if (!pl.stop) {
        p->used = mark;
        pl.start = nullptr;
    }
    return pl;
}

void prof_launch_end(int phase, hipStream_t st, const ProfLaunch& pl, double bytes, double flops)
{
    Profiler* p = g_prof;
    if (!p || p->phase != phase || capturing(st)) return;
    p->seen += 1;
    if (!pl.start) return;
    p->launches += 1;
    p->bytes += bytes;
    p->flops += flops;
}

void* prof_suspend()
{
    Profiler* p = g_prof;
    g_prof = nullptr;
    return p;
}

void prof_resume(void* saved) { g_prof = static_cast<Profiler*>(saved); }

Profiler* prof_start(int phase, int stride, size_t reserve)
{
    Profiler* p = new Profiler;
    p->phase = phase;
    p->stride = stride < 1 ? 1 : stride;
    p->pool.reserve(reserve);
    for (size_t q = 0; q < reserve; ++q) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) break;
        p->pool.push_back(e);
    }
    g_prof = p;
    return p;
}

bool prof_stop(Profiler* p, int64_t* launches, int64_t* seen, double* ms, double* bytes, double* flops)
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
    if (seen) *seen = p->seen;
    if (ms) *ms = total;
    if (bytes) *bytes = p->bytes;
    if (flops) *flops = p->flops;
    for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
    delete p;
    return ok;
}

}  // namespace kgev
