// Scheduling core of the serving loop: admission of eigensolve requests by
// device-memory footprint and by free execution slots, in arrival order, as
// earlier requests complete (continuous batching at request granularity).
// Optionally (max_bypass > 0) a request behind a head that does not fit the
// remaining budget may start first if it fits, at most max_bypass times per
// head, so that small requests fill memory a large one is waiting for without
// the large one ever starving.
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

    // Bypass limit (0: strict arrival order); takes effect at the next step.
    void set_max_bypass(int k) { max_bypass_ = k > 0 ? k : 0; }
    int max_bypass() const { return max_bypass_; }

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
    // remaining budget; when the head does not fit, the earliest later
    // request that does is admitted instead, while the head has been passed
    // fewer than max_bypass times.  Returns the number of requests that
    // changed state.
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
            size_t pick = 0;
            if (used_ + queue_.front()->footprint > budget_) {
                if (passed_ >= max_bypass_) break;          // keep arrival order
                for (size_t q = 1; q < queue_.size(); ++q)
                    if (used_ + queue_[q]->footprint <= budget_) { pick = q; break; }
                if (pick == 0) break;
            }
            int slot = -1;
            for (size_t s = 0; s < slot_busy_.size(); ++s)
                if (!slot_busy_[s]) { slot = (int)s; break; }
            if (slot < 0) break;
            Req* r = queue_[pick];
            queue_.erase(queue_.begin() + (ptrdiff_t)pick);
            if (pick == 0)
                passed_ = 0;        // a new head
            else
                ++passed_;
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
    int max_bypass_ = 0;
    int passed_ = 0;                // times the current head has been passed
    std::vector<Req*> slot_busy_;
    std::deque<Req*> queue_;
};

}  // namespace kgev
