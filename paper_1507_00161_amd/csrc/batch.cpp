// batch.cpp - grouped launches of the H_eff products of several contexts.
#include "batch.h"

#include <algorithm>
#include <cstring>

namespace dm {

namespace {
constexpr size_t kTableBytes = (size_t)4 << 20;
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

Batch::Batch(int device) {
    char buf[512] = {0};
    if (dmrgdev::ctx_create(device, nullptr, &dev_, buf, sizeof(buf))) {
        err_ = buf;
        dev_ = nullptr;
        return;
    }
    d_table_ = dmrgdev::alloc(dev_, kTableBytes);
    if (!d_table_) {
        err_ = "device allocation of the batch tables failed";
        dmrgdev::ctx_destroy(dev_);
        dev_ = nullptr;
        return;
    }
    table_cap_ = kTableBytes;
    for (auto& e : group_end_) {
        e = dmrgdev::xevent_create(dev_);
        if (!e) {
            err_ = "event creation for the batch failed";
            for (auto& f : group_end_) dmrgdev::xevent_destroy(f);
            dmrgdev::release(dev_, d_table_);
            dmrgdev::ctx_destroy(dev_);
            dev_ = nullptr;
            return;
        }
    }
    launcher_ = std::thread([this] { loop(); });
}

Batch::~Batch() {
    if (!dev_) return;
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_launcher_.notify_all();
    launcher_.join();
    dmrgdev::sync(dev_);
    for (auto& e : group_end_) dmrgdev::xevent_destroy(e);
    dmrgdev::release(dev_, d_table_);
    dmrgdev::ctx_destroy(dev_);
}

std::string Batch::error() {
    std::lock_guard<std::mutex> lk(mu_);
    return err_;
}

int Batch::run(HeffRequest& r) {
    std::unique_lock<std::mutex> lk(mu_);
    if (failed_) return 1;
    r.launched = false;
    pending_.push_back(&r);
    cv_launcher_.notify_one();
    cv_.wait(lk, [&] { return r.launched || failed_; });
    return r.launched ? 0 : 1;
}

void Batch::loop() {
    dmrgdev::bind(dev_);
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
        cv_launcher_.wait(lk, [&] { return stop_ || failed_ || !pending_.empty(); });
        if (failed_ || (pending_.empty() && stop_)) return;
        std::vector<HeffRequest*> reqs;
        reqs.swap(pending_);
        lk.unlock();
        int rc = launch(reqs);
        if (!rc) rc = dmrgdev::xevent_record(dev_, group_end_[ngroups_ & 1]);
        lk.lock();
        if (rc) {
            if (err_.empty()) err_ = dmrgdev::last_error(dev_);
            failed_ = true;
            cv_.notify_all();
            return;
        }
        for (auto* r : reqs) r->launched = true;
        ++launches_;
        products_ += (int64_t)reqs.size();
        cv_.notify_all();
        // This group stays queued behind the previous one; wait for that one
        // to end, so that products arriving meanwhile gather into the next.
        if (ngroups_++ > 0) {
            lk.unlock();
            rc = dmrgdev::xevent_sync(dev_, group_end_[(ngroups_ - 2) & 1]);
            lk.lock();
            if (rc) {
                if (err_.empty()) err_ = dmrgdev::last_error(dev_);
                failed_ = true;
                cv_.notify_all();
                return;
            }
        }
    }
}

// One group: per operand precision, the batch stream waits for every
// product's input; each phase is one grouped GEMM launch over the plans of
// all products (and one grouped split-K reduction); every product's `done`
// event is recorded.  The descriptor tables of the whole group are laid out
// in one host image and uploaded with one copy (stream-ordered after the
// previous group's kernels, which have read their tables by then).
int Batch::launch(std::vector<HeffRequest*>& reqs) {
    auto fail = [&](const std::string& m) {
        std::lock_guard<std::mutex> lk(mu_);
        err_ = m;
        return 1;
    };
    std::vector<int> precs;
    for (auto* r : reqs)
        if (std::find(precs.begin(), precs.end(), r->ab_prec) == precs.end()) precs.push_back(r->ab_prec);
    struct Launch {
        int prec, cp, ph, n, total;
        size_t plans, prefix;
        bool red;
    };
    std::vector<Launch> ls;
    table_.clear();
    auto put = [&](const void* src, size_t bytes) {
        const size_t off = table_.size();
        table_.resize(off + align256(bytes));
        std::memcpy(table_.data() + off, src, bytes);
        return off;
    };
    for (int prec : precs) {
        std::vector<HeffRequest*> grp;
        for (auto* r : reqs)
            if (r->ab_prec == prec) grp.push_back(r);
        for (int ph = 0; ph < 3; ++ph) {
            std::vector<dmrgdev::PlanDesc> pd;
            std::vector<int32_t> pre{0};
            std::vector<dmrgdev::RedDesc> rd;
            std::vector<int32_t> rpre{0};
            for (auto* r : grp) {
                if (r->nwg[ph] > 0) {
                    pd.push_back(r->plan[ph]);
                    pre.push_back(pre.back() + r->nwg[ph]);
                }
                if (r->nreds[ph] > 0) {
                    rd.push_back(r->red[ph]);
                    rpre.push_back(rpre.back() + r->nreds[ph]);
                }
            }
            const int cp = grp[0]->c_prec[ph];
            if (!pd.empty()) {
                const size_t a = put(pd.data(), pd.size() * sizeof(pd[0]));
                const size_t b = put(pre.data(), pre.size() * sizeof(int32_t));
                ls.push_back({prec, cp, ph, (int)pd.size(), pre.back(), a, b, false});
            }
            if (!rd.empty()) {
                const size_t a = put(rd.data(), rd.size() * sizeof(rd[0]));
                const size_t b = put(rpre.data(), rpre.size() * sizeof(int32_t));
                ls.push_back({prec, cp, ph, (int)rd.size(), rpre.back(), a, b, true});
            }
        }
    }
    if (table_.size() > table_cap_) return fail("batch descriptor tables exceed their buffer");
    for (auto* r : reqs)
        if (dmrgdev::xevent_wait(dev_, r->ready)) return fail(dmrgdev::last_error(dev_));
    if (!table_.empty() && dmrgdev::h2d_async(dev_, d_table_, table_.data(), table_.size()))
        return fail(dmrgdev::last_error(dev_));
    char* base = (char*)d_table_;
    for (const Launch& l : ls) {
        const int32_t* prefix = (const int32_t*)(base + l.prefix);
        int rc;
        if (l.red) {
            rc = dmrgdev::gemm_reduce_multi(dev_, l.cp, (const dmrgdev::RedDesc*)(base + l.plans), prefix, l.n, l.total);
        } else {
            const int kind = l.ph == 0 ? dmrgdev::GK_HEFF_Z : l.ph == 1 ? dmrgdev::GK_HEFF_Y : dmrgdev::GK_OTHER;
            rc = dmrgdev::gemm_multi(dev_, l.prec, l.cp, (const dmrgdev::PlanDesc*)(base + l.plans), prefix, l.n,
                                     l.total, kind);
        }
        if (rc) return fail(dmrgdev::last_error(dev_));
    }
    for (auto* r : reqs)
        if (dmrgdev::xevent_record(dev_, r->done)) return fail(dmrgdev::last_error(dev_));
    return 0;
}

}  // namespace dm
