// batch.h - H_eff products of several contexts advanced together.
//
// While dmrg_sweep_many runs, every context submits its H_eff products here
// instead of launching them on its own stream.  A launcher thread takes all
// products pending at once and launches them together on the batch's stream:
// each GEMM phase (and each split-K reduction) of all of them is one grouped
// launch of the persistent kernel over the concatenation of their plans.
// At most two groups are on the device at a time (one running, one queued
// behind it); products that arrive meanwhile form the next group, so the
// grouping follows the load and no product waits for a timeout.
#pragma once
#include <condition_variable>
#include <cstdint>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "device.h"

namespace dm {

// One product of one context: plans of the three phases (ntasks 0 = none),
// their reductions, and the precisions.  `ready` is recorded on the context
// stream when the product's input is there; `done` is recorded on the batch
// stream after its launches, and the context stream must wait for it.
struct HeffRequest {
    int ab_prec = 0;
    int c_prec[3] = {0, 0, 0};
    dmrgdev::PlanDesc plan[3];
    dmrgdev::RedDesc red[3];
    int nwg[3] = {0, 0, 0};
    int nreds[3] = {0, 0, 0};
    void* ready = nullptr;
    void* done = nullptr;
    bool launched = false;
};

class Batch {
public:
    explicit Batch(int device);
    ~Batch();
    bool ok() const { return dev_ != nullptr; }
    std::string error();
    // Queue the product and return once it is launched (its `done` event
    // recorded); 0 on success.
    int run(HeffRequest& r);
    int64_t launches() const { return launches_; }
    int64_t products() const { return products_; }

private:
    dmrgdev::Ctx* dev_ = nullptr;
    std::string err_;
    std::mutex mu_;
    std::condition_variable cv_, cv_launcher_;
    std::vector<HeffRequest*> pending_;
    int64_t launches_ = 0, products_ = 0;
    bool failed_ = false, stop_ = false;
    std::thread launcher_;
    // device copy of the descriptor table of one launch, and its host image
    void* d_table_ = nullptr;
    size_t table_cap_ = 0;
    std::vector<char> table_;
    // end of the last two groups on the batch stream
    void* group_end_[2] = {nullptr, nullptr};
    int64_t ngroups_ = 0;
    void loop();
    int launch(std::vector<HeffRequest*>& reqs);
};

}  // namespace dm
