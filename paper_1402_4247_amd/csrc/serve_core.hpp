// Scheduling core of the serving loop: admission of eigensolve requests by
// device-memory footprint and by free execution slots, in arrival order, as
// earlier requests complete (continuous batching at request granularity).
// Plain C++ with no HIP dependency: the executor that actually runs a request
// is a template parameter, so the policy can be exercised on the host with a
// stand-in executor.
//
// Executor interface:
//   size_t footprint(const Req&)            device bytes the request needs
//   bool   start(Req&, int slot)            begin running on `slot`; false = failed to start
//   bool   finished(Req&, int slot)         non-blocking completion test
//   void   finish(Req&, int slot)           collect results, release resources
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <vector>

namespace kgev {

enum ReqState { RQ_QUEUED = 0, RQ_RUNNING = 1, RQ_DONE = 2 };

template <typename Req, typename Exec>
class ServeCore {
public:
    ServeCore(size_t budget, int slots) : budget_(budget), slot_busy_(slots > 0 ? slots : 1, nullptr) {}

    size_t budget() const { return budget_; }
    size_t in_use() const { return used_; }
    int running() const
    {
        int r = 0;
        for (Req* q : slot_busy_) r += (q != nullptr);
        return r;
    }
    size_t queued() const { return queue_.size(); }

    // Queue a request.  One whose footprint can never fit the budget is
    // rejected at once (returns false and leaves it untouched).
    bool submit(Req* r, Exec& ex)
    {
        r->footprint = ex.footprint(*r);
        if (r->footprint > budget_) return false;
        r->state = RQ_QUEUED;
        queue_.push_back(r);
        return true;
    }

    // One scheduling pass: retire finished requests, then admit queued ones
    // in arrival order while a slot is free and the head request fits the
    // remaining budget.  Returns the number of requests that changed state.
    int step(Exec& ex)
    {
        int changed = 0;
        for (size_t s = 0; s < slot_busy_.size(); ++s) {
            Req* r = slot_busy_[s];
            if (r && ex.finished(*r, (int)s)) {
                ex.finish(*r, (int)s);
                used_ -= r->footprint;
                r->state = RQ_DONE;
                slot_busy_[s] = nullptr;
                ++changed;
            }
        }
        while (!queue_.empty()) {
            Req* r = queue_.front();
            if (used_ + r->footprint > budget_) break;     // head-of-line: keep arrival order
            int slot = -1;
            for (size_t s = 0; s < slot_busy_.size(); ++s)
                if (!slot_busy_[s]) { slot = (int)s; break; }
            if (slot < 0) break;
            queue_.pop_front();
            used_ += r->footprint;
            r->state = RQ_RUNNING;
            slot_busy_[slot] = r;
            if (!ex.start(*r, slot)) {
                // failed to start: the request completes with its error set by
                // the executor; its resources are returned at once
                ex.finish(*r, slot);
                used_ -= r->footprint;
                r->state = RQ_DONE;
                slot_busy_[slot] = nullptr;
            }
            ++changed;
        }
        return changed;
    }

private:
    size_t budget_;
    size_t used_ = 0;
    std::vector<Req*> slot_busy_;
    std::deque<Req*> queue_;
};

}  // namespace kgev
