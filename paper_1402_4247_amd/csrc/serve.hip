// Serving loop (kgev_server_*): requests of mixed order n and k-point count
// are admitted as execution slots and device memory free up, each admitted
// request runs the batched per-k solve on its own HIP stream with a
// stream-ordered workspace allocation, so requests admitted while others are
// running overlap with them on the device.  Admission is in arrival order and
// by the request's workspace footprint against the server's HBM budget.
// One worker thread owns the device work; submit/poll/wait may be called from
// any thread.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "serve_core.hpp"
#include "../../include/kgev.h"

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct ServeReq {
    uint64_t ticket = 0;
    kgev_request rq{};
    kgev_opts opts{};
    size_t footprint = 0;
    std::atomic<int> state{kgev::RQ_QUEUED};
    size_t work_bytes = 0;
    void* dwork = nullptr;           // workspace + status words
    int32_t* hstatus = nullptr;      // pinned copy of the per-k status words
    hipEvent_t done = nullptr;
    kgev_status status = KGEV_OK;
    int64_t bad_k = -1;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

struct Exec {
    kgev_ctx* ctx = nullptr;
    std::vector<hipStream_t> streams;

    static size_t status_off(size_t work) { return (work + 255) & ~(size_t)255; }

    size_t footprint(const ServeReq& r)
    {
        const size_t w = kgev_workspace_bytes(r.rq.n, r.rq.nk, &r.opts);
        return status_off(w) + sizeof(int32_t) * (size_t)r.rq.nk;
    }

    bool start(ServeReq& r, int slot)
    {
        hipStream_t st = streams[slot];
        r.t_admit = now_s();
        r.work_bytes = kgev_workspace_bytes(r.rq.n, r.rq.nk, &r.opts);
        if (hipMallocAsync(&r.dwork, r.footprint, st) != hipSuccess) {
            r.dwork = nullptr;
            r.status = KGEV_ENOMEM;
            return false;
        }
        int32_t* dst = reinterpret_cast<int32_t*>(static_cast<char*>(r.dwork) + status_off(r.work_bytes));
        kgev_status s = kgev_solve_k_device(ctx, r.rq.dH, r.rq.dS, r.rq.n, r.rq.ld, r.rq.nk, r.rq.dw, r.rq.dC,
                                            r.rq.ldc, r.dwork, r.work_bytes, dst, &r.opts, st);
        if (s == KGEV_OK && hipMemcpyAsync(r.hstatus, dst, sizeof(int32_t) * r.rq.nk, hipMemcpyDeviceToHost, st) != hipSuccess)
            s = KGEV_EDEVICE;
        if (s == KGEV_OK && hipEventRecord(r.done, st) != hipSuccess) s = KGEV_EDEVICE;
        if (s != KGEV_OK) {
            r.status = s;
            return false;
        }
        return true;
    }

    bool finished(ServeReq& r, int)
    {
        const hipError_t e = hipEventQuery(r.done);
        if (e == hipErrorNotReady) return false;
        if (e != hipSuccess) r.status = KGEV_EDEVICE;
        return true;
    }

    void finish(ServeReq& r, int slot)
    {
        if (r.dwork) (void)hipFreeAsync(r.dwork, streams[slot]);
        r.dwork = nullptr;
        if (r.status == KGEV_OK) {
            for (int64_t q = 0; q < r.rq.nk; ++q)
                if (r.hstatus[q] != 0) {
                    r.status = r.hstatus[q];
                    r.bad_k = q;
                    break;
                }
        }
        r.t_done = now_s();
    }
};

}  // namespace

struct kgev_server {
    int device = 0;
    Exec ex;
    kgev::ServeCore<ServeReq, Exec>* core = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<ServeReq*> incoming;
    std::unordered_map<uint64_t, ServeReq*> reqs;
    uint64_t next = 1;
    bool stop = false;
    std::atomic<int> bypass{0};     // applied to the core by the worker
    std::thread worker;
};

namespace {

void worker_main(kgev_server* s)
{
    (void)hipSetDevice(s->device);
    for (;;) {
        std::vector<ServeReq*> add;
        bool stopping;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->incoming.empty() && s->core->running() == 0 && s->core->queued() == 0 && !s->stop)
                s->cv.wait(lk, [&] { return !s->incoming.empty() || s->stop; });
            add.assign(s->incoming.begin(), s->incoming.end());
            s->incoming.clear();
            stopping = s->stop;
        }
        bool changed = false;
        for (ServeReq* r : add) {
            if (!s->core->submit(r, s->ex)) {
                r->status = KGEV_ENOMEM;     // can never fit the budget
                r->t_admit = r->t_done = now_s();
                r->state = kgev::RQ_DONE;
                changed = true;
            }
        }
        s->core->set_max_bypass(s->bypass.load());
        if (s->core->step(s->ex) > 0) changed = true;
        if (changed) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->cv.notify_all();
        }
        if (stopping && s->core->running() == 0 && s->core->queued() == 0) break;
        if (!changed) std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

}  // namespace

extern "C" {

kgev_status kgev_server_create(kgev_server** out, int device, size_t hbm_budget, int32_t max_slots)
{
    if (!out) return -1;
    *out = nullptr;
    if (max_slots < 1 || max_slots > 64) return -4;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return KGEV_EDEVICE;
    if (device < 0 || device >= count) return -2;
    if (hipSetDevice(device) != hipSuccess) return KGEV_EDEVICE;
    if (hbm_budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return KGEV_EDEVICE;
        const size_t reserve = (size_t)4 << 30;
        hbm_budget = fr > 2 * reserve ? fr - reserve : fr / 2;
    }
    kgev_server* s = new kgev_server;
    s->device = device;
    if (kgev_create(&s->ex.ctx, device) != KGEV_OK) {
        delete s;
        return KGEV_EDEVICE;
    }
    for (int q = 0; q < max_slots; ++q) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : s->ex.streams) (void)hipStreamDestroy(x);
            kgev_destroy(s->ex.ctx);
            delete s;
            return KGEV_EDEVICE;
        }
        s->ex.streams.push_back(st);
    }
    s->core = new kgev::ServeCore<ServeReq, Exec>(hbm_budget, max_slots);
    s->worker = std::thread(worker_main, s);
    *out = s;
    return KGEV_OK;
}

kgev_status kgev_server_set_bypass(kgev_server* s, int32_t max_bypass)
{
    if (!s) return -1;
    if (max_bypass < 0) return -2;
    s->bypass.store(max_bypass);
    s->cv.notify_all();
    return KGEV_OK;
}

kgev_status kgev_server_submit(kgev_server* s, const kgev_request* rq, uint64_t* ticket)
{
    if (!s) return -1;
    if (!rq) return -2;
    if (!ticket) return -3;
    if (rq->n < 1 || rq->nk < 1 || rq->ld < rq->n || !rq->dH || !rq->dS || !rq->dw) return -2;
    kgev_opts o;
    kgev_opts_default(&o);
    o.precision = rq->precision;
    o.want_vectors = rq->dC ? 1 : 0;
    if (o.want_vectors && rq->ldc < rq->n) return -2;
    if (o.precision != KGEV_PREC_FP64 && o.precision != KGEV_PREC_FP32_REFINE) return -2;
    ServeReq* r = new ServeReq;
    r->rq = *rq;
    r->opts = o;
    if (hipHostMalloc((void**)&r->hstatus, sizeof(int32_t) * rq->nk, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&r->done, hipEventDisableTiming) != hipSuccess) {
        if (r->hstatus) (void)hipHostFree(r->hstatus);
        delete r;
        return KGEV_EDEVICE;
    }
    r->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->ticket = s->next++;
        s->reqs[r->ticket] = r;
        s->incoming.push_back(r);
        *ticket = r->ticket;
    }
    s->cv.notify_all();
    return KGEV_OK;
}

kgev_status kgev_server_poll(kgev_server* s, uint64_t ticket, int32_t* done)
{
    if (!s) return -1;
    if (!done) return -3;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return -2;
    *done = it->second->state.load() == kgev::RQ_DONE ? 1 : 0;
    return KGEV_OK;
}

kgev_status kgev_server_wait(kgev_server* s, uint64_t ticket, kgev_result* res)
{
    if (!s) return -1;
    if (!res) return -3;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return -2;
    ServeReq* r = it->second;
    s->cv.wait(lk, [&] { return r->state.load() == kgev::RQ_DONE; });
    res->status = r->status;
    res->bad_k = r->bad_k;
    res->t_submit = r->t_submit;
    res->t_admit = r->t_admit;
    res->t_done = r->t_done;
    res->footprint = r->footprint;
    s->reqs.erase(it);
    lk.unlock();
    (void)hipEventDestroy(r->done);
    (void)hipHostFree(r->hstatus);
    delete r;
    return KGEV_OK;
}

void kgev_server_destroy(kgev_server* s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto& kv : s->reqs) {
        (void)hipEventDestroy(kv.second->done);
        (void)hipHostFree(kv.second->hstatus);
        delete kv.second;
    }
    for (hipStream_t x : s->ex.streams) (void)hipStreamDestroy(x);
    kgev_destroy(s->ex.ctx);
    delete s->core;
    delete s;
}

}  // extern "C"
