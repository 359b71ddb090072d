// Host-only harness for the serving scheduler: drives kgev::ServeCore (the
// product's admission policy) with a stand-in executor whose requests finish
// after a given number of scheduling steps.  Test infrastructure only.
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "serve_core.hpp"

namespace {

struct FakeReq {
    int id = 0;
    size_t want = 0;        // declared footprint
    int steps_left = 0;     // steps until it finishes once started
    bool fail_start = false;
    size_t footprint = 0;
    int state = 0;
    int slot = -1;
    int start_seq = -1;     // order in which requests were started
    int failed = 0;
};

struct FakeExec {
    int started = 0;
    int max_running = 0, running = 0;
    size_t peak_bytes = 0, bytes = 0;
    size_t footprint(const FakeReq& r) { return r.want; }
    bool start(FakeReq& r, int slot)
    {
        r.slot = slot;
        r.start_seq = started++;
        if (r.fail_start) { r.failed = 1; return false; }
        ++running;
        bytes += r.want;
        if (running > max_running) max_running = running;
        if (bytes > peak_bytes) peak_bytes = bytes;
        return true;
    }
    bool finished(FakeReq& r, int) { return --r.steps_left <= 0; }
    void finish(FakeReq& r, int)
    {
        if (!r.failed) { --running; bytes -= r.want; }
    }
};

struct Harness {
    FakeExec ex;
    kgev::ServeCore<FakeReq, FakeExec> core;
    std::vector<FakeReq*> reqs;
    Harness(size_t budget, int slots) : core(budget, slots) {}
    ~Harness() { for (FakeReq* r : reqs) delete r; }
};

}  // namespace

extern "C" {

void* sh_create(uint64_t budget, int slots) { return new Harness(budget, slots); }
void sh_destroy(void* h) { delete static_cast<Harness*>(h); }

int sh_submit(void* hp, uint64_t footprint, int steps, int fail_start)
{
    Harness* h = static_cast<Harness*>(hp);
    FakeReq* r = new FakeReq;
    r->id = (int)h->reqs.size();
    r->want = footprint;
    r->steps_left = steps;
    r->fail_start = fail_start != 0;
    h->reqs.push_back(r);
    return h->core.submit(r, h->ex) ? r->id : -1;
}

void sh_set_bypass(void* hp, int k) { static_cast<Harness*>(hp)->core.set_max_bypass(k); }
int sh_step(void* hp) { Harness* h = static_cast<Harness*>(hp); return h->core.step(h->ex); }
int sh_state(void* hp, int id) { return static_cast<Harness*>(hp)->reqs[id]->state; }
int sh_start_seq(void* hp, int id) { return static_cast<Harness*>(hp)->reqs[id]->start_seq; }
int sh_failed(void* hp, int id) { return static_cast<Harness*>(hp)->reqs[id]->failed; }
int sh_max_running(void* hp) { return static_cast<Harness*>(hp)->ex.max_running; }
uint64_t sh_peak_bytes(void* hp) { return static_cast<Harness*>(hp)->ex.peak_bytes; }
uint64_t sh_in_use(void* hp) { return static_cast<Harness*>(hp)->core.in_use(); }
int sh_running(void* hp) { return static_cast<Harness*>(hp)->core.running(); }

}  // extern "C"
