// engine.cpp - host control of the two-site DMRG hot path.
//
// Structure of one two-site step at bond b (sites b, b+1 explicit):
//   S = L_b * s_b and E = s_{b+1} * R_{b+2} are "enlarged" blocks whose states
//   are grouped by (base-block sector, site occupation).  Their operators are
//   linear combinations of base-block operators times 2x2 site operators
//   (blocking), written here as formula lists and executed on the device as
//   scaled block copies.  H_eff psi is a sum of terms op(A) psi op(B)^T over
//   S- and E-operators (complementary operators carry the two-body sums),
//   executed as two grouped GEMM launches.  The lowest eigenpair is found by
//   Davidson; the S (or E) reduced density matrix is diagonalised per sector,
//   the D largest weights are kept, the operators renormalised (U^T O U), and
//   the state is carried to the next bond as the next initial guess.
#include "engine.h"

#include "batch.h"

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <numeric>
#include <queue>
#include <set>
#include <sstream>
#include <thread>

namespace dm {

using dmrgdev::DiagTask;
using dmrgdev::DiagTerm;
using dmrgdev::GemmChunk;
using dmrgdev::GemmTask;
using dmrgdev::LcTask;
using dmrgdev::LcTerm;

// ---------------------------------------------------------------- hashing
// SplitMix64 (Steele, Lea, Flood 2014) chained over the key fields.
static inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static uint64_t hkey(std::initializer_list<int64_t> vals) {
    uint64_t h = 0;
    for (int64_t v : vals) h = splitmix64(h ^ (uint64_t)v);
    return h;
}
static inline double u01(uint64_t h) { return (double)(h >> 11) * (1.0 / 9007199254740992.0); }

static double now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ----------------------------------------------------------------- memory
Buf& Buf::operator=(Buf&& o) noexcept {
    if (this != &o) {
        reset();
        eng = o.eng;
        p = o.p;
        bytes = o.bytes;
        o.p = nullptr;
        o.bytes = 0;
    }
    return *this;
}
void Buf::reset() {
    if (p && eng) eng->dfree(p, bytes);
    p = nullptr;
    bytes = 0;
}

// size classes 2^k (1 + j/8): at most 12.5% padding
static size_t size_class(size_t b) {
    if (b <= 4096) return 4096;
    int k = 63 - __builtin_clzll((unsigned long long)b);
    size_t step = (size_t)1 << (k - 3);
    return (b + step - 1) / step * step;
}

void* Engine::dalloc(size_t bytes) {
    // 64 bytes of slack past every block: the 16-byte reads of a GEMM
    // operand's last elements never reach the end of an allocation
    const size_t c = size_class(bytes + 64);
    // a cached block of this class, or of one of the next two classes
    auto it = cache_.lower_bound(c);
    if (it != cache_.end() && it->first <= c + c / 4) {
        void* p = it->second;
        const size_t s = it->first;
        cache_.erase(it);
        cached_ -= s;
        live_[p] = s;
        return p;
    }
    if (opt_.mem_cap_bytes && mem_used_ + c > opt_.mem_cap_bytes) trim_cache(0);
    if (opt_.mem_cap_bytes && mem_used_ + c > opt_.mem_cap_bytes) return nullptr;
    void* p = dmrgdev::alloc(dev_, c);
    if (!p && cached_) {
        trim_cache(0);
        p = dmrgdev::alloc(dev_, c);
    }
    if (!p) return nullptr;
    mem_used_ += c;
    live_[p] = c;
    return p;
}
void Engine::dfree(void* p, size_t) {
    auto it = live_.find(p);
    if (it == live_.end()) return;
    const size_t s = it->second;
    live_.erase(it);
    if (dying_) {
        dmrgdev::release(dev_, p);
        mem_used_ -= s;
        return;
    }
    cache_.emplace(s, p);
    cached_ += s;
    // bound the cache: release the largest blocks beyond 16 GiB
    const size_t limit = (size_t)16 << 30;
    if (cached_ > limit) trim_cache(limit / 2);
}
// release cached blocks, largest first, until at most `keep` bytes stay cached
void Engine::trim_cache(size_t keep) {
    while (cached_ > keep && !cache_.empty()) {
        auto it = std::prev(cache_.end());
        dmrgdev::release(dev_, it->second);
        cached_ -= it->first;
        mem_used_ -= it->first;
        cache_.erase(it);
    }
}
dmrg_status Engine::alloc_buf(Buf& b, size_t bytes) {
    b.reset();
    b.p = dalloc(bytes);
    if (!b.p) {
        std::ostringstream s;
        s << "device allocation of " << bytes << " bytes failed (in use " << mem_used_ << ")";
        return fail(DMRG_ERR_OUT_OF_MEMORY, s.str());
    }
    b.eng = this;
    b.bytes = bytes;
    return DMRG_OK;
}
template <class T> dmrg_status Engine::upload(Buf& b, const std::vector<T>& v) {
    dmrg_status st = alloc_buf(b, std::max<size_t>(v.size() * sizeof(T), 8));
    if (st) return st;
    if (!v.empty() && dmrgdev::h2d_async(dev_, b.p, v.data(), v.size() * sizeof(T)))
        return fail(DMRG_ERR_DEVICE, dmrgdev::last_error(dev_));
    return DMRG_OK;
}

Engine::~Engine() {
    dmrgdev::graph_destroy(graph_exec_);
    dmrgdev::xevent_destroy(ev_ready_);
    dmrgdev::xevent_destroy(ev_done_);
    dying_ = true;   // buffers released from here on go straight back to the device
    cur_.reset();
    L_.clear();
    R_.clear();
    trim_cache(0);
}

#define TRY(x)                        \
    do {                              \
        dmrg_status _s = (x);         \
        if (_s < 0) return _s;        \
    } while (0)
#define DEV(x)                                                         \
    do {                                                               \
        if ((x) != 0) return fail(DMRG_ERR_DEVICE, dmrgdev::last_error(dev_)); \
    } while (0)

// ------------------------------------------------------ GEMM plan builder
// Output blocks with their chunk lists are collected first; `finish_plan`
// then tiles them (64 x 64) and splits a tile's chunk list over several
// work-groups when the plan has fewer tiles than the chip has room for
// (split-K into partial tiles, reduced in a fixed order by a second kernel).
struct GB {
    struct OB {
        int cbuf;
        int64_t coff;
        int ldc, M, Nn, beta;
        int64_t cb, ce;
    };
    std::vector<OB> obs;
    std::vector<GemmChunk> chunks;
    // per chunk: output columns that can be nonzero (the rest of the block's
    // width is multiplied by cleared operand columns); empty = all
    std::vector<int> nuse;
    int64_t cb = 0;
    double flops = 0.0, issued = 0.0, elems = 0.0;
    void begin() { cb = (int64_t)chunks.size(); }
    void chunk(double alpha, int abuf, int64_t aoff, int lda, bool atr, int bbuf, int64_t boff, int ldb,
               bool btr, int K) {
        GemmChunk c;
        c.alpha = alpha;
        c.a_off = aoff;
        c.b_off = boff;
        c.lda = lda;
        c.ldb = ldb;
        c.K = K;
        c.a_buf = (uint8_t)abuf;
        c.b_buf = (uint8_t)bbuf;
        c.a_trans = atr;
        c.b_trans = btr;
        chunks.push_back(c);
    }
    void end(int cbuf, int64_t coff, int ldc, int M, int Nn, int beta) {
        int64_t ce = (int64_t)chunks.size();
        for (int64_t x = cb; x < ce; ++x) {
            const int nu = x < (int64_t)nuse.size() ? nuse[x] : Nn;
            flops += 2.0 * M * nu * chunks[x].K;
            issued += 2.0 * M * Nn * chunks[x].K;
            elems += (double)chunks[x].K * (M + nu);
        }
        elems += (double)M * Nn * (beta ? 2 : 1);
        obs.push_back({cbuf, coff, ldc, M, Nn, beta, cb, ce});
    }
};

dmrg_status Engine::run_gemm(int prec, BufTable bufs, const GemmPlan& p, int cprec, int kind, void* partials,
                             int ev_start, int ev_stop) {
    if (cprec < 0) cprec = prec == dmrgdev::P_BF16 ? dmrgdev::P_F32 : prec;
    if (p.ntasks == 0) {
        if (ev_start >= 0) DEV(dmrgdev::event_record(dev_, ev_start));
        if (ev_stop >= 0) DEV(dmrgdev::event_record(dev_, ev_stop));
        return DMRG_OK;
    }
    if (p.nslots) {
        if (partials) {
            bufs[dmrgdev::kPartialBuf] = partials;
        } else {
            TRY(ensure_partials(p.nslots));
            bufs[dmrgdev::kPartialBuf] = partial_.p;
        }
    }
    dmrgdev::Sched sc;
    sc.wg_off = p.wg_off;
    sc.nwg = p.nwg;
    sc.nfull = p.nfull;
    sc.ntasks = p.ntasks;
    DEV(dmrgdev::gemm(dev_, prec, cprec, bufs.data(), p.tasks, sc, p.chunks, kind,
                      ev_start, ev_stop));
    if (p.nreds)
        DEV(dmrgdev::gemm_reduce(dev_, cprec, bufs.data(), p.reds, p.nreds));
    return DMRG_OK;
}

dmrg_status Engine::ensure_partials(int64_t slots) {
    size_t need = (size_t)slots * dmrgdev::kTileM * dmrgdev::kTileN * sizeof(double);
    if (partial_.bytes >= need) return DMRG_OK;
    return alloc_buf(partial_, need);
}

// Static schedule of a persistent GEMM launch.  Estimated task cost: its K
// slices plus a fixed start/epilogue overhead.  Output blocks (all their
// tiles and split-K parts, which are consecutive in `tasks`) are dealt to the
// 8 XCDs, each onto the least-loaded XCD, so that the tiles sharing A rows
// or B columns share one L2; blocks larger than 1/64 of the launch are dealt
// tile by tile.  When work-groups get few tasks (under 16 each), units and
// then tasks go longest-first, each task to its XCD's least-loaded
// work-group; with more tasks, both dealings keep plan order and tasks go
// round-robin over the XCD's work-groups (no sorting).  Tasks without chunks
// (pure clears) are moved behind all others.  The task vector is reordered in place: work-group
// w = 8 j + x runs [wg_off[w], wg_off[w+1]).
static void schedule_tasks(const GB& g, std::vector<GemmTask>& tasks, const std::vector<int32_t>& owner,
                           std::vector<int32_t>& wg_off, int& nwg, int& nfull, bool parallel) {
    const int64_t n = (int64_t)tasks.size();
    std::vector<float> cost(n, 0.f);
    double total = 0.0;
    int64_t nf = 0;
    for (int64_t t = 0; t < n; ++t) {
        const GemmTask& tk = tasks[t];
        if (tk.chunk_begin == tk.chunk_end) continue;
        double c = 64.0;
        for (int32_t k = tk.chunk_begin; k < tk.chunk_end; ++k) c += 32.0 * ((g.chunks[k].K + 31) / 32) + 8.0;
        cost[t] = (float)c;
        total += c;
        ++nf;
    }
    nfull = (int)nf;
    const int gw = (int)std::max<int64_t>(1, std::min<int64_t>(128, (nf + 7) / 8));
    nwg = 8 * gw;
    // units: [begin, end) runs of one output block, or single tasks of big blocks
    struct Unit {
        double c;
        int64_t b, e;
    };
    std::vector<Unit> units;
    for (int64_t t = 0; t < n;) {
        int64_t e = t;
        double c = 0.0;
        while (e < n && owner[e] == owner[t]) c += cost[e++];
        if (c <= total / 64.0) {
            if (c > 0.0) units.push_back({c, t, e});
        } else {
            for (int64_t u = t; u < e; ++u)
                if (cost[u] > 0.f) units.push_back({cost[u], u, u + 1});
        }
        t = e;
    }
    const bool lpt = nf < 16 * (int64_t)nwg;
    if (lpt)
        std::sort(units.begin(), units.end(),
                  [](const Unit& a, const Unit& b) { return a.c != b.c ? a.c > b.c : a.b < b.b; });
    std::vector<int8_t> xcd_of(n, -1);
    std::array<double, 8> xload{};
    std::array<int64_t, 8> xcount{};
    for (const Unit& u : units) {
        int best = 0;
        for (int x = 1; x < 8; ++x)
            if (xload[x] < xload[best]) best = x;
        xload[best] += u.c;
        for (int64_t t = u.b; t < u.e; ++t)
            if (cost[t] > 0.f) {
                xcd_of[t] = (int8_t)best;
                ++xcount[best];
            }
    }
    // tasks of each XCD, in dealing order
    std::vector<int64_t> xoff(9, 0);
    for (int x = 0; x < 8; ++x) xoff[x + 1] = xoff[x] + xcount[x];
    std::vector<int64_t> order(nf);
    {
        std::vector<int64_t> fp(xoff.begin(), xoff.end() - 1);
        if (lpt) {
            for (const Unit& u : units)
                for (int64_t t = u.b; t < u.e; ++t)
                    if (xcd_of[t] >= 0) order[fp[xcd_of[t]]++] = t;
        } else {
            for (int64_t t = 0; t < n; ++t)
                if (xcd_of[t] >= 0) order[fp[xcd_of[t]]++] = t;
        }
    }
    // per XCD: each task onto its least-loaded work-group.  With few tasks per
    // work-group the tasks go largest first (LPT); with many, in dealing order
    // (list scheduling), so that work-groups running at the same time work on
    // neighbouring tiles, which share operands in the XCD's L2, while the
    // loads still end within about one task of each other.
    std::vector<int32_t> wg_of(n, -1);
    typedef std::pair<double, int> QE;
    auto cmp = [](const QE& a, const QE& b) { return a > b; };   // min-heap on (load, j)
    // the XCDs' dealings touch disjoint tasks: one host thread each for large plans
    auto deal = [&](int x) {
        std::vector<QE> heap;
        auto b = order.begin() + xoff[x], e = order.begin() + xoff[x + 1];
        if (lpt)
            std::sort(b, e, [&](int64_t p, int64_t q) { return cost[p] != cost[q] ? cost[p] > cost[q] : p < q; });
        for (int j = 0; j < gw; ++j) heap.push_back({0.0, j});
        std::make_heap(heap.begin(), heap.end(), cmp);
        for (auto it = b; it != e; ++it) {
            std::pop_heap(heap.begin(), heap.end(), cmp);
            QE& q = heap.back();
            wg_of[*it] = 8 * q.second + x;
            q.first += cost[*it];
            std::push_heap(heap.begin(), heap.end(), cmp);
        }
    };
    if (parallel && nf >= 8192) {
        std::vector<std::thread> th;
        for (int x = 1; x < 8; ++x) th.emplace_back(deal, x);
        deal(0);
        for (auto& t : th) t.join();
    } else {
        for (int x = 0; x < 8; ++x) deal(x);
    }
    // counting sort by work-group; within a work-group, tasks keep dealing order
    wg_off.assign(nwg + 1, 0);
    for (int64_t t = 0; t < n; ++t)
        if (wg_of[t] >= 0) ++wg_off[wg_of[t] + 1];
    for (int w = 0; w < nwg; ++w) wg_off[w + 1] += wg_off[w];
    std::vector<GemmTask> out(n);
    std::vector<int32_t> fillp(wg_off.begin(), wg_off.end() - 1);
    for (int64_t t : order) out[fillp[wg_of[t]]++] = tasks[t];
    int64_t z = nf;
    for (int64_t t = 0; t < n; ++t)
        if (cost[t] == 0.f) out[z++] = tasks[t];
    tasks.swap(out);
}

// Host part of a plan: tiles, split-K parts and the schedule (no device
// calls, so two plans can be prepared on two threads).
struct PlanHost {
    std::vector<GemmTask> tasks;
    std::vector<dmrgdev::RedTask> reds;
    std::vector<int32_t> wg_off;
};
static void plan_host(const GB& g, GemmPlan& p, PlanHost& h, bool parallel = true) {
    using dmrgdev::kTileM;
    using dmrgdev::kTileN;
    std::vector<GemmTask>& tasks = h.tasks;
    std::vector<int32_t> owner;   // scheduling unit of each task
    int32_t unit = 0;
    std::vector<dmrgdev::RedTask>& reds = h.reds;
    // total work in K units, tile by tile
    double work = 0.0;
    int64_t ntiles = 0;
    for (const auto& ob : g.obs) {
        double kk = 0.0;
        for (int64_t c = ob.cb; c < ob.ce; ++c) kk += g.chunks[c].K;
        int64_t nt = (int64_t)((ob.M + kTileM - 1) / kTileM) * ((ob.Nn + kTileN - 1) / kTileN);
        work += kk * nt;
        ntiles += nt;
    }
    // split-K parts: enough tasks for about 8 per persistent work-group, so
    // that the static schedule balances; no part below 512 K
    const double target = 8192.0;
    const double kper = std::max(work / target, 512.0);
    int64_t slot = 0;
    for (const auto& ob : g.obs) {
        double kk = 0.0;
        for (int64_t c = ob.cb; c < ob.ce; ++c) kk += g.chunks[c].K;
        int parts = (int)std::min(64.0, std::max(1.0, std::ceil(kk / kper)));
        if (ob.ce - ob.cb < 2) parts = 1;
        // chunk ranges of the parts (balanced by K)
        std::vector<std::pair<int64_t, int64_t>> ranges;
        if (parts == 1) {
            ranges.push_back({ob.cb, ob.ce});
        } else {
            double run = 0.0;
            int64_t start = ob.cb;
            int q = 1;
            for (int64_t c = ob.cb; c < ob.ce; ++c) {
                run += g.chunks[c].K;
                if (run >= kk * q / parts && c + 1 < ob.ce) {
                    ranges.push_back({start, c + 1});
                    start = c + 1;
                    ++q;
                }
            }
            if (start < ob.ce) ranges.push_back({start, ob.ce});
        }
        // tiles of the block; with split-K, tasks are listed part by part so
        // that the tiles reading one chunk range (the same A rows and B
        // columns) form one scheduling unit
        std::vector<GemmTask> tiles;
        for (int m0 = 0; m0 < ob.M; m0 += kTileM)
            for (int n0 = 0; n0 < ob.Nn; n0 += kTileN) {
                GemmTask t{};
                t.ldc = ob.ldc;
                t.m0 = m0;
                t.n0 = n0;
                t.mt = std::min(kTileM, ob.M - m0);
                t.nt = std::min(kTileN, ob.Nn - n0);
                tiles.push_back(t);
            }
        if (ranges.size() == 1) {
            for (GemmTask t : tiles) {
                t.c_off = ob.coff;
                t.chunk_begin = (int32_t)ranges[0].first;
                t.chunk_end = (int32_t)ranges[0].second;
                t.c_buf = (uint8_t)ob.cbuf;
                t.beta = (uint8_t)ob.beta;
                t.c_local = 0;
                tasks.push_back(t);
                owner.push_back(unit);
            }
            ++unit;
            continue;
        }
        const int64_t nparts = (int64_t)ranges.size();
        for (size_t q = 0; q < tiles.size(); ++q) {
            const GemmTask& t = tiles[q];
            dmrgdev::RedTask r{};
            r.dst_off = ob.coff + (int64_t)t.m0 * ob.ldc + t.n0;
            r.ld = ob.ldc;
            r.mt = t.mt;
            r.nt = t.nt;
            r.slot0 = (int32_t)(slot + (int64_t)q * nparts);
            r.nslots = (int32_t)nparts;
            r.dst_buf = (uint8_t)ob.cbuf;
            r.beta = (uint8_t)ob.beta;
            reds.push_back(r);
        }
        for (int64_t pq = 0; pq < nparts; ++pq) {
            for (size_t q = 0; q < tiles.size(); ++q) {
                GemmTask u = tiles[q];
                u.c_off = (slot + (int64_t)q * nparts + pq) * (int64_t)kTileM * kTileN;
                u.chunk_begin = (int32_t)ranges[pq].first;
                u.chunk_end = (int32_t)ranges[pq].second;
                u.c_buf = (uint8_t)dmrgdev::kPartialBuf;
                u.beta = 0;
                u.c_local = 1;
                tasks.push_back(u);
                owner.push_back(unit);
            }
            ++unit;
        }
        slot += (int64_t)tiles.size() * nparts;
    }
    (void)ntiles;
    schedule_tasks(g, tasks, owner, h.wg_off, p.nwg, p.nfull, parallel);
    p.ntasks = (int)tasks.size();
    p.nreds = (int)reds.size();
    p.nslots = slot;
    p.nchunks = (int64_t)g.chunks.size();
    p.flops = g.flops;
    p.issued = g.issued;
    p.elems = g.elems;
}

// The four lists of a plan go up in one copy, laid out at 256-byte offsets
// in one device block.
static dmrg_status plan_upload(Engine& e, const GB& g, GemmPlan& p, const PlanHost& h) {
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t bt = h.tasks.size() * sizeof(GemmTask), bw = h.wg_off.size() * sizeof(int32_t),
                 br = h.reds.size() * sizeof(dmrgdev::RedTask), bc = g.chunks.size() * sizeof(GemmChunk);
    const size_t ot = 0, ow = al(bt), orr = ow + al(bw), oc = orr + al(br);
    std::vector<char> img(std::max<size_t>(oc + al(bc), 8));
    if (bt) std::memcpy(img.data() + ot, h.tasks.data(), bt);
    if (bw) std::memcpy(img.data() + ow, h.wg_off.data(), bw);
    if (br) std::memcpy(img.data() + orr, h.reds.data(), br);
    if (bc) std::memcpy(img.data() + oc, g.chunks.data(), bc);
    dmrg_status st = e.upload(p.dev, img);
    if (st) return st;
    char* base = p.dev.as<char>();
    p.tasks = bt ? reinterpret_cast<GemmTask*>(base + ot) : nullptr;
    p.wg_off = bw ? reinterpret_cast<int32_t*>(base + ow) : nullptr;
    p.reds = br ? reinterpret_cast<dmrgdev::RedTask*>(base + orr) : nullptr;
    p.chunks = bc ? reinterpret_cast<GemmChunk*>(base + oc) : nullptr;
    return DMRG_OK;
}

static dmrg_status finish_plan(Engine& e, GB& g, GemmPlan& p) {
    PlanHost h;
    plan_host(g, p, h, e.host_threads(1 << 20) > 1);
    return plan_upload(e, g, p, h);
}

// Both plans of one H_eff term group: the host parts on two threads.
static dmrg_status finish_plans(Engine& e, GB& g1, GemmPlan& p1, GB& g2, GemmPlan& p2) {
    PlanHost h1, h2;
    const bool par = e.host_threads(1 << 20) > 1;
    std::thread t([&] { plan_host(g1, p1, h1, par); });
    plan_host(g2, p2, h2, par);
    t.join();
    dmrg_status st = plan_upload(e, g1, p1, h1);
    if (st) return st;
    return plan_upload(e, g2, p2, h2);
}

// ------------------------------------------------ linear-combination builder
struct LB {
    std::vector<LcTask> tasks;
    std::vector<LcTerm> terms;
    void block(int dbuf, int64_t doff, int rows, int cols, const std::vector<LcTerm>& ts) {
        int32_t t0 = (int32_t)terms.size();
        terms.insert(terms.end(), ts.begin(), ts.end());
        int32_t t1 = (int32_t)terms.size();
        for (int r0 = 0; r0 < rows; r0 += dmrgdev::kLcTile)
            for (int c0 = 0; c0 < cols; c0 += dmrgdev::kLcTile) {
                LcTask t;
                t.dst_off = doff;
                t.ld = cols;
                t.r0 = r0;
                t.c0 = c0;
                t.mt = std::min(dmrgdev::kLcTile, rows - r0);
                t.nt = std::min(dmrgdev::kLcTile, cols - c0);
                t.t_begin = t0;
                t.t_end = t1;
                t.buf = (uint8_t)dbuf;
                t.pad0 = t.pad1 = t.pad2 = 0;
                tasks.push_back(t);
            }
    }
    dmrg_status run(Engine& e, double* const* bufs) {
        if (tasks.empty()) return DMRG_OK;
        Buf dt, dterm;
        dmrg_status st = e.upload(dt, tasks);
        if (st) return st;
        st = e.upload(dterm, terms);
        if (st) return st;
        if (dmrgdev::lincomb(e.dev(), bufs, dt.as<LcTask>(), (int)tasks.size(), dterm.as<LcTerm>()))
            return e.fail(DMRG_ERR_DEVICE, dmrgdev::last_error(e.dev()));
        // the task lists go back to the stream-ordered cache on return: later
        // users are ordered after this kernel, so no wait is needed
        return DMRG_OK;
    }
};

// --------------------------------------------------------------- reach
Engine::Reach Engine::make_reach(int a, int b) const {
    Reach r;
    int maxm = 0;
    for (int i = 0; i < N_; ++i) maxm += std::abs(tm0_.empty() ? 0 : delta_[i].tm);
    r.off = maxm;
    r.width = 2 * maxm + 1;
    int cp = 0, cn = 0;
    for (int i = a; i < b; ++i) (delta_[i].np ? cp : cn)++;
    r.p.assign(cp + 1, std::vector<char>(r.width, 0));
    r.n.assign(cn + 1, std::vector<char>(r.width, 0));
    r.p[0][r.off] = 1;
    r.n[0][r.off] = 1;
    int kp = 0, kn = 0;
    for (int i = a; i < b; ++i) {
        auto& tab = delta_[i].np ? r.p : r.n;
        int& k = delta_[i].np ? kp : kn;
        int m = delta_[i].tm;
        for (int c = k; c >= 0; --c)
            for (int t = 0; t < r.width; ++t)
                if (tab[c][t] && t + m >= 0 && t + m < r.width) tab[c + 1][t + m] = 1;
        ++k;
    }
    return r;
}

bool Engine::reachable(const Reach& r, const QN& q) const {
    if (q.np < 0 || q.nn < 0 || q.np >= (int)r.p.size() || q.nn >= (int)r.n.size()) return false;
    const auto& P = r.p[q.np];
    const auto& Nn = r.n[q.nn];
    for (int tp = 0; tp < r.width; ++tp) {
        if (!P[tp]) continue;
        int tn = q.tm - (tp - r.off) + r.off;
        if (tn >= 0 && tn < r.width && Nn[tn]) return true;
    }
    return false;
}

// --------------------------------------------------------------- loading
dmrg_status Engine::load(int n, const int32_t* species, const int32_t* two_m, const double* eps,
                         const double* V, int n_p, int n_n, int two_M) {
    if (n < 1 || n > 64 || !species || !two_m || !eps || !V)
        return fail(DMRG_ERR_ARG, "n_sites must be in 1..64 and all arrays non-null");
    cur_.reset();
    L_.clear();
    R_.clear();
    psi_.reset();
    psi1_.reset();
    init_ = false;
    loaded_ = false;
    cideas_ = false;
    meas_valid_ = false;
    have_energy_ = false;
    have_prev_sweep_ = false;
    sweeps_done_ = 0;
    for (int i = 0; i < n; ++i) {
        if (species[i] != 0 && species[i] != 1) return fail(DMRG_ERR_ARG, "species must be 0 or 1");
        if (!std::isfinite(eps[i])) return fail(DMRG_ERR_HAMILTONIAN, "eps is not finite");
    }
    size_t n4 = (size_t)n * n * n * n;
    double vmax = 0.0;
    for (size_t x = 0; x < n4; ++x) {
        if (!std::isfinite(V[x])) return fail(DMRG_ERR_HAMILTONIAN, "V is not finite");
        vmax = std::max(vmax, std::fabs(V[x]));
    }
    double tol = 1e-12 * std::max(vmax, 1e-300);
    auto at = [&](int i, int j, int k, int l) { return V[(((size_t)i * n + j) * n + k) * n + l]; };
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k)
                for (int l = 0; l < n; ++l) {
                    double v = at(i, j, k, l);
                    bool bad = std::fabs(v + at(j, i, k, l)) > tol || std::fabs(v + at(i, j, l, k)) > tol ||
                               std::fabs(v - at(k, l, i, j)) > tol;
                    const char* why = "antisymmetry / (ij)<->(kl) symmetry";
                    if (!bad && std::fabs(v) > tol) {
                        bool mok = two_m[i] + two_m[j] == two_m[k] + two_m[l];
                        int a = species[i] + species[j], b = species[k] + species[l];
                        if (!mok || a != b) {
                            bad = true;
                            why = "selection rule (2M or charge not conserved)";
                        }
                    }
                    if (bad) {
                        std::ostringstream s;
                        s << "V violates " << why << " at (i,j,k,l) = (" << i << "," << j << "," << k
                          << "," << l << ")";
                        return fail(DMRG_ERR_HAMILTONIAN, s.str());
                    }
                }
    N_ = n;
    sp0_.assign(species, species + n);
    tm0_.assign(two_m, two_m + n);
    eps0_.assign(eps, eps + n);
    V0_.assign(V, V + n4);
    T_ = QN(n_p, n_n, two_M);
    // target reachable from all sites?
    order_.clear();
    delta_.assign(n, QN());
    for (int i = 0; i < n; ++i) delta_[i] = species[i] == 0 ? QN(1, 0, two_m[i]) : QN(0, 1, two_m[i]);
    Reach all = make_reach(0, n);
    if (!reachable(all, T_)) return fail(DMRG_ERR_TARGET, "target (n_p, n_n, 2M) is not reachable");
    loaded_ = true;
    return DMRG_OK;
}

dmrg_status Engine::set_order(const int32_t* ordering) {
    std::vector<int> ord(N_);
    if (ordering) {
        std::vector<char> seen(N_, 0);
        for (int i = 0; i < N_; ++i) {
            int s = ordering[i];
            if (s < 0 || s >= N_ || seen[s]) return fail(DMRG_ERR_ARG, "ordering is not a permutation");
            seen[s] = 1;
            ord[i] = s;
        }
    } else {
        std::iota(ord.begin(), ord.end(), 0);
    }
    if (init_ && ord == order_) return DMRG_OK;
    order_ = ord;
    meas_valid_ = false;
    eps_.assign(N_, 0.0);
    V_.assign((size_t)N_ * N_ * N_ * N_, 0.0);
    delta_.assign(N_, QN());
    for (int a = 0; a < N_; ++a) {
        int s = ord[a];
        eps_[a] = eps0_[s];
        delta_[a] = sp0_[s] == 0 ? QN(1, 0, tm0_[s]) : QN(0, 1, tm0_[s]);
    }
    for (int a = 0; a < N_; ++a)
        for (int b = 0; b < N_; ++b)
            for (int c = 0; c < N_; ++c)
                for (int d = 0; d < N_; ++d)
                    V_[(((size_t)a * N_ + b) * N_ + c) * N_ + d] =
                        V0_[(((size_t)ord[a] * N_ + ord[b]) * N_ + ord[c]) * N_ + ord[d]];
    pre_.clear();
    for (int b = 0; b <= N_; ++b) pre_.push_back(make_reach(0, b));
    init_ = false;
    return DMRG_OK;
}

std::unique_ptr<Stored> Engine::vacuum(char side, int lo) {
    auto v = std::make_unique<Stored>();
    v->side = side;
    v->lo = lo;
    v->hi = lo;
    v->normal = true;
    v->basis.add(QN(), 1);
    Op h;
    h.dq = QN();
    h.par = 0;
    h.blk.push_back({0, 0, v->ops.alloc_block(1, 1), 1, 1});
    h.index();
    v->ops.add({'H', 0, 0}, std::move(h));
    if (alloc_buf(v->ops.pool, v->ops.size * sizeof(double))) return nullptr;
    if (dmrgdev::fill(dev_, v->ops.pool.d(), v->ops.size, 0.0)) return nullptr;
    v->has_cfg = true;
    v->cfg.push_back({0});
    return v;
}

// ============================================================== blocking
// A blocked operator is sum_terms (sum_refs coef * op_ref(base)) x site_op.
enum SiteOp { S_I = 0, S_CD = 1, S_C = 2, S_N = 3 };
static int site_par(int s) { return (s == S_CD || s == S_C) ? 1 : 0; }
static int site_dsig(int s) { return s == S_CD ? 1 : (s == S_C ? -1 : 0); }
// nonzero (sigma_out, sigma_in) elements with value 1
static const std::vector<std::pair<int, int>>& site_elems(int s) {
    static const std::vector<std::pair<int, int>> e_i = {{0, 0}, {1, 1}}, e_cd = {{1, 0}}, e_c = {{0, 1}},
                                                   e_n = {{1, 1}};
    switch (s) {
        case S_I: return e_i;
        case S_CD: return e_cd;
        case S_C: return e_c;
        default: return e_n;
    }
}
struct Ref {
    int op;        // index into the base op set
    bool trans;
    double coef;
};
struct FTerm {
    int site;
    bool ident = false;     // base part is the identity (times icoef)
    double icoef = 0.0;
    std::vector<Ref> refs;
};
using Formula = std::vector<FTerm>;

struct Lin {
    std::vector<Ref> refs;
};

// helpers returning a base-block operator (or a combination of them)
struct FormulaCtx {
    const Engine& e;
    const Stored& B;
    void add(Lin& l, const Key& k, double c, bool tr) const {
        if (c == 0.0) return;
        int x = B.ops.find(k);
        if (x >= 0) l.refs.push_back({x, tr, c});
    }
    Lin one(const Key& k, double c = 1.0, bool tr = false) const {
        Lin l;
        add(l, k, c, tr);
        return l;
    }
    // P^L_kl = sum_{i<j in L} V_ijkl c+_i c+_j
    Lin PL(int k, int l) const {
        Lin r;
        if (!B.normal) return one({'P', k, l});
        for (int i = B.lo; i < B.hi; ++i)
            for (int j = i + 1; j < B.hi; ++j) add(r, {'A', i, j}, e.V(i, j, k, l), false);
        return r;
    }
    // Q^L_jl = sum_{i,k in L} V_ijkl c+_i c_k
    Lin QL(int j, int l) const {
        Lin r;
        if (!B.normal) return j <= l ? one({'Q', j, l}) : one({'Q', l, j}, 1.0, true);
        for (int i = B.lo; i < B.hi; ++i)
            for (int k = B.lo; k < B.hi; ++k) {
                if (i <= k) add(r, {'B', i, k}, e.V(i, j, k, l), false);
                else add(r, {'B', k, i}, e.V(i, j, k, l), true);
            }
        return r;
    }
    // P^R_ij = sum_{k<l in R} V_ijkl c_l c_k
    Lin PR(int i, int j) const {
        Lin r;
        if (!B.normal) return one({'P', i, j});
        for (int k = B.lo; k < B.hi; ++k)
            for (int l = k + 1; l < B.hi; ++l) add(r, {'A', k, l}, e.V(i, j, k, l), true);
        return r;
    }
    // Q^R_ik = sum_{j,l in R} V_ijkl c+_j c_l
    Lin QR(int i, int k) const {
        Lin r;
        if (!B.normal) return i <= k ? one({'Q', i, k}) : one({'Q', k, i}, 1.0, true);
        for (int j = B.lo; j < B.hi; ++j)
            for (int l = B.lo; l < B.hi; ++l) {
                if (j <= l) add(r, {'B', j, l}, e.V(i, j, k, l), false);
                else add(r, {'B', l, j}, e.V(i, j, k, l), true);
            }
        return r;
    }
};

static void push(Formula& f, int site, const Lin& l, double scale = 1.0) {
    if (l.refs.empty()) return;
    FTerm t;
    t.site = site;
    for (auto r : l.refs) {
        r.coef *= scale;
        t.refs.push_back(r);
    }
    f.push_back(std::move(t));
}
static void push_ident(Formula& f, int site, double c) {
    if (c == 0.0) return;
    FTerm t;
    t.site = site;
    t.ident = true;
    t.icoef = c;
    f.push_back(std::move(t));
}

// formulas for S = L * s (s = L.hi) at bond s
static std::vector<std::pair<Key, Formula>> left_formulas(const Engine& e, const Stored& L) {
    FormulaCtx F{e, L};
    const int s = L.hi, N = e.N();
    std::vector<std::pair<Key, Formula>> out;
    // H_S = H_L + eps_s n_s + Q^L_ss n_s + R^L_s c_s + (R^L_s c_s)^+,
    // (R c_s)^+ = c+_s R^+ = -R^+ c+_s
    {
        Formula f;
        push(f, S_I, F.one({'H', 0, 0}));
        push_ident(f, S_N, e.eps(s));
        push(f, S_N, F.QL(s, s));
        push(f, S_C, F.one({'R', s, 0}));
        push(f, S_CD, F.one({'R', s, 0}, -1.0, true));
        out.push_back({{'H', 0, 0}, f});
    }
    for (int i = L.lo; i < L.hi; ++i) {
        Formula f;
        push(f, S_I, F.one({'C', i, 0}));
        out.push_back({{'C', i, 0}, f});
    }
    {
        Formula f;
        push_ident(f, S_CD, 1.0);
        out.push_back({{'C', s, 0}, f});
    }
    if (e.measuring()) {
        // occupation operators of every S site, for the orbital correlations
        for (int i = L.lo; i < L.hi; ++i) {
            Formula f;
            push(f, S_I, F.one({'N', i, 0}));
            if (!f.empty()) out.push_back({{'N', i, 0}, f});
        }
        Formula f;
        push_ident(f, S_N, 1.0);
        out.push_back({{'N', s, 0}, f});
    }
    // R^S_l = R^L_l + Q^L_sl c+_s - P^L_sl c_s - (sum_i V_issl c+_i) n_s
    for (int l = s + 1; l < N; ++l) {
        Formula f;
        push(f, S_I, F.one({'R', l, 0}));
        push(f, S_CD, F.QL(s, l));
        push(f, S_C, F.PL(s, l), -1.0);
        Lin cn;
        for (int i = L.lo; i < L.hi; ++i) F.add(cn, {'C', i, 0}, -e.V(i, s, s, l), false);
        push(f, S_N, cn);
        out.push_back({{'R', l, 0}, f});
    }
    if (e.normal_S(s)) {
        for (int i = L.lo; i < L.hi; ++i) {
            for (int j = i + 1; j < L.hi; ++j) {
                Formula f;
                push(f, S_I, F.one({'A', i, j}));
                out.push_back({{'A', i, j}, f});
            }
            Formula fa;
            push(fa, S_CD, F.one({'C', i, 0}));
            out.push_back({{'A', i, s}, fa});
            for (int k = i; k < L.hi; ++k) {
                Formula f;
                push(f, S_I, F.one({'B', i, k}));
                out.push_back({{'B', i, k}, f});
            }
            Formula fb;
            push(fb, S_C, F.one({'C', i, 0}));
            out.push_back({{'B', i, s}, fb});
        }
        Formula f;
        push_ident(f, S_N, 1.0);
        out.push_back({{'B', s, s}, f});
    } else {
        for (int k = s + 1; k < N; ++k)
            for (int l = k + 1; l < N; ++l) {
                // P^S_kl = P^L_kl + sum_i V_iskl c+_i c+_s
                Formula f;
                push(f, S_I, F.PL(k, l));
                Lin cs;
                for (int i = L.lo; i < L.hi; ++i) F.add(cs, {'C', i, 0}, e.V(i, s, k, l), false);
                push(f, S_CD, cs);
                out.push_back({{'P', k, l}, f});
            }
        for (int j = s + 1; j < N; ++j)
            for (int l = j; l < N; ++l) {
                // Q^S_jl = Q^L_jl + sum_i V_ijsl c+_i c_s - sum_k V_sjkl c_k^+.. c+_s + V_sjsl n_s
                Formula f;
                push(f, S_I, F.QL(j, l));
                Lin a, b;
                for (int i = L.lo; i < L.hi; ++i) F.add(a, {'C', i, 0}, e.V(i, j, s, l), false);
                for (int k = L.lo; k < L.hi; ++k) F.add(b, {'C', k, 0}, -e.V(s, j, k, l), true);
                push(f, S_C, a);
                push(f, S_CD, b);
                push_ident(f, S_N, e.V(s, j, s, l));
                out.push_back({{'Q', j, l}, f});
            }
    }
    return out;
}

// formulas for E = s * R (s = R.lo - 1) at bond s - 1
static std::vector<std::pair<Key, Formula>> right_formulas(const Engine& e, const Stored& R) {
    FormulaCtx F{e, R};
    const int s = R.lo - 1;
    std::vector<std::pair<Key, Formula>> out;
    // H_E = H_R + eps_s n_s + n_s Q^R_ss + c+_s R^R_s + (c+_s R^R_s)^+,
    // (c+_s R)^+ = R^+ c_s = -c_s R^+
    {
        Formula f;
        push(f, S_I, F.one({'H', 0, 0}));
        push_ident(f, S_N, e.eps(s));
        push(f, S_N, F.QR(s, s));
        push(f, S_CD, F.one({'R', s, 0}));
        push(f, S_C, F.one({'R', s, 0}, -1.0, true));
        out.push_back({{'H', 0, 0}, f});
    }
    {
        Formula f;
        push_ident(f, S_CD, 1.0);
        out.push_back({{'C', s, 0}, f});
    }
    for (int j = R.lo; j < R.hi; ++j) {
        Formula f;
        push(f, S_I, F.one({'C', j, 0}));
        out.push_back({{'C', j, 0}, f});
    }
    // R^E_i = R^R_i + c+_s P^R_is + c_s Q^R_is - n_s sum_l V_issl c_l
    for (int i = 0; i < s; ++i) {
        Formula f;
        push(f, S_I, F.one({'R', i, 0}));
        push(f, S_CD, F.PR(i, s));
        push(f, S_C, F.QR(i, s));
        Lin cn;
        for (int l = R.lo; l < R.hi; ++l) F.add(cn, {'C', l, 0}, -e.V(i, s, s, l), true);
        push(f, S_N, cn);
        out.push_back({{'R', i, 0}, f});
    }
    if (!e.normal_S(s - 1)) {
        for (int l = R.lo; l < R.hi; ++l) {
            Formula fa, fb;
            push(fa, S_CD, F.one({'C', l, 0}));
            push(fb, S_CD, F.one({'C', l, 0}, 1.0, true));
            out.push_back({{'A', s, l}, fa});
            out.push_back({{'B', s, l}, fb});
        }
        for (int k = R.lo; k < R.hi; ++k) {
            for (int l = k + 1; l < R.hi; ++l) {
                Formula f;
                push(f, S_I, F.one({'A', k, l}));
                out.push_back({{'A', k, l}, f});
            }
            for (int l = k; l < R.hi; ++l) {
                Formula f;
                push(f, S_I, F.one({'B', k, l}));
                out.push_back({{'B', k, l}, f});
            }
        }
        Formula f;
        push_ident(f, S_N, 1.0);
        out.push_back({{'B', s, s}, f});
    } else {
        for (int i = 0; i < s; ++i)
            for (int j = i + 1; j < s; ++j) {
                // P^E_ij = P^R_ij - sum_l V_ijsl c_s c_l
                Formula f;
                push(f, S_I, F.PR(i, j));
                Lin cl;
                for (int l = R.lo; l < R.hi; ++l) F.add(cl, {'C', l, 0}, -e.V(i, j, s, l), true);
                push(f, S_C, cl);
                out.push_back({{'P', i, j}, f});
            }
        for (int i = 0; i < s; ++i)
            for (int k = i; k < s; ++k) {
                // Q^E_ik = Q^R_ik + V_isks n_s + sum_l V_iskl c+_s c_l - sum_j V_ijks c_s c+_j
                Formula f;
                push(f, S_I, F.QR(i, k));
                push_ident(f, S_N, e.V(i, s, k, s));
                Lin a, b;
                for (int l = R.lo; l < R.hi; ++l) F.add(a, {'C', l, 0}, e.V(i, s, k, l), true);
                for (int j = R.lo; j < R.hi; ++j) F.add(b, {'C', j, 0}, -e.V(i, j, k, s), false);
                push(f, S_CD, a);
                push(f, S_C, b);
                out.push_back({{'Q', i, k}, f});
            }
    }
    return out;
}

// Build the enlarged block (sub-sectors of base sectors x site occupation),
// keeping merged sectors whose quantum numbers are in `allowed` (sorted), and
// its operators from the formulas, executed as scaled block copies.
dmrg_status Engine::enlarge(const Stored& base, char side, const std::vector<QN>& allowed, Enl& en,
                            OpSet& ops) {
    LB lb;
    std::string why;
    if (!enlarge_plan(base, side, allowed, en, ops, lb, why)) return fail(DMRG_ERR_DEVICE, why);
    return enlarge_run(base, ops, lb);
}

// Host part of `enlarge`: no device calls and no change to the engine, so the
// two blocks of a bond can be planned on two threads.  Returns false (with a
// message) on an internal inconsistency.
bool Engine::enlarge_plan(const Stored& base, char side, const std::vector<QN>& allowed, Enl& en, OpSet& ops,
                          LB& lb, std::string& why) const {
    const int s = side == 'L' ? base.hi : base.lo - 1;
    en = Enl();
    en.side = side;
    en.site = s;
    en.dsite = delta_[s];
    std::set<QN> allow(allowed.begin(), allowed.end());
    std::map<QN, std::array<int, 2>> parts;   // merged q -> base sector per sigma
    for (int sg = 0; sg < 2; ++sg)
        for (size_t b = 0; b < base.basis.q.size(); ++b) {
            QN q = sg ? base.basis.q[b] + delta_[s] : base.basis.q[b];
            if (!allow.count(q)) continue;
            auto it = parts.find(q);
            if (it == parts.end()) it = parts.insert({q, {-1, -1}}).first;
            it->second[sg] = (int)b;
        }
    for (auto& kv : parts) {
        int m = (int)en.mq.size();
        en.midx[kv.first] = m;
        en.mq.push_back(kv.first);
        std::array<int, 2> ms = {-1, -1};
        int off = 0;
        for (int sg = 0; sg < 2; ++sg) {
            int b = kv.second[sg];
            if (b < 0) continue;
            Sub sb{m, b, sg, off, base.basis.d[b], kv.first};
            off += sb.dim;
            ms[sg] = (int)en.sub.size();
            en.sub_of[{b, sg}] = (int)en.sub.size();
            if (en.sub_tab.size() < (size_t)(2 * b + 2)) en.sub_tab.resize(2 * b + 2, -1);
            en.sub_tab[2 * b + sg] = (int)en.sub.size();
            en.sub.push_back(sb);
        }
        en.md.push_back(off);
        en.msub.push_back(ms);
    }
    // operators
    auto formulas = side == 'L' ? left_formulas(*this, base) : right_formulas(*this, base);
    ops = OpSet();
    const int nbase = (int)base.basis.q.size();
    const int64_t nsub = (int64_t)en.sub.size();
    // Per formula, its dq, parity and contributions (out sub, in sub, term):
    // formed on several host threads, each formula on its own, then laid out
    // in formula order below (block offsets and copies are those of a
    // serial pass).
    struct FPlan {
        QN dq;
        int par = 0;
        std::vector<std::pair<int64_t, LcTerm>> contrib;
    };
    std::vector<FPlan> fplans(formulas.size());
    auto plan_formula = [&](size_t fi) {
        const Formula& f = formulas[fi].second;
        if (f.empty()) return;
        FPlan& fp = fplans[fi];
        std::vector<std::pair<int64_t, LcTerm>>& contrib = fp.contrib;
        // dq and parity from the first term
        QN bdq;
        int bpar = 0;
        const FTerm& t0 = f[0];
        if (!t0.ident) {
            const Op& o = base.ops.ops[t0.refs[0].op];
            bdq = t0.refs[0].trans ? -o.dq : o.dq;
            bpar = o.par;
        }
        int ds = site_dsig(t0.site);
        fp.dq = ds == 1 ? bdq + delta_[s] : (ds == -1 ? bdq - delta_[s] : bdq);
        fp.par = (bpar + site_par(t0.site)) % 2;
        // contributions (out sub, in sub, term), walking each referenced
        // operator's blocks (a stored operator has at most one block per input
        // sector); grouped by (out, in) with a stable sort, which keeps the
        // term order of the formula inside a group
        for (const FTerm& t : f) {
            const int tpar = t.ident ? 0 : base.ops.ops[t.refs[0].op].par;
            const auto& els = site_elems(t.site);
            auto sign_of = [&](int b_in, int sigma) {
                if (side == 'L') return (site_par(t.site) && (base.basis.q[b_in].n() & 1)) ? -1.0 : 1.0;
                return (tpar && sigma) ? -1.0 : 1.0;
            };
            if (t.ident) {
                for (int b_in = 0; b_in < nbase; ++b_in)
                    for (const auto& el : els) {
                        const int i_in = en.find_sub(b_in, el.second), i_out = en.find_sub(b_in, el.first);
                        if (i_in < 0 || i_out < 0) continue;
                        LcTerm lt{};
                        lt.coef = t.icoef * sign_of(b_in, el.second);
                        lt.ident = 1;
                        contrib.push_back({(int64_t)i_out * nsub + i_in, lt});
                    }
                continue;
            }
            for (const Ref& r : t.refs) {
                const Op& o = base.ops.ops[r.op];
                for (const Blk& bk : o.blk) {
                    const int b_in = r.trans ? bk.out : bk.in;
                    const int b_out = r.trans ? bk.in : bk.out;
                    for (const auto& el : els) {
                        const int i_in = en.find_sub(b_in, el.second), i_out = en.find_sub(b_out, el.first);
                        if (i_in < 0 || i_out < 0) continue;
                        LcTerm lt{};
                        lt.coef = r.coef * sign_of(b_in, el.second);
                        lt.src_off = bk.off;
                        lt.ld = bk.cols;
                        lt.trans = r.trans;
                        lt.buf = 0;
                        contrib.push_back({(int64_t)i_out * nsub + i_in, lt});
                    }
                }
            }
        }
        std::stable_sort(contrib.begin(), contrib.end(),
                         [](const std::pair<int64_t, LcTerm>& x, const std::pair<int64_t, LcTerm>& y) {
                             return x.first < y.first;
                         });
    };
    {
        std::atomic<size_t> next(0);
        auto run = [&] {
            for (size_t fi = next++; fi < formulas.size(); fi = next++) plan_formula(fi);
        };
        // the two enlarged blocks are planned side by side: half the threads each
        const int nth = std::max(1, host_threads((int64_t)formulas.size()) / 2);
        std::vector<std::thread> pool;
        for (int t = 1; t < nth; ++t) pool.emplace_back(run);
        run();
        for (auto& th : pool) th.join();
    }
    std::vector<LcTerm> terms;
    for (size_t fi = 0; fi < formulas.size(); ++fi) {
        const FPlan& fp = fplans[fi];
        const std::vector<std::pair<int64_t, LcTerm>>& contrib = fp.contrib;
        if (contrib.empty()) continue;
        Op op;
        op.dq = fp.dq;
        op.par = fp.par;
        for (size_t g0 = 0; g0 < contrib.size();) {
            size_t g1 = g0;
            terms.clear();
            while (g1 < contrib.size() && contrib[g1].first == contrib[g0].first) terms.push_back(contrib[g1++].second);
            const int i_out = (int)(contrib[g0].first / nsub), i_in = (int)(contrib[g0].first % nsub);
            const Sub& so = en.sub[i_out];
            const Sub& si = en.sub[i_in];
            if (so.q != si.q + fp.dq) {
                why = "internal: inconsistent blocking formula";
                return false;
            }
            Blk bk{i_out, i_in, ops.alloc_block(so.dim, si.dim), so.dim, si.dim};
            op.blk.push_back(bk);
            lb.block(1, bk.off, bk.rows, bk.cols, terms);
            g0 = g1;
        }
        op.index();
        ops.add(formulas[fi].first, std::move(op));
    }
    return true;
}

// Device part of `enlarge`: the operator pool and the block copies.
dmrg_status Engine::enlarge_run(const Stored& base, OpSet& ops, LB& lb) {
    TRY(alloc_buf(ops.pool, std::max<int64_t>(ops.size, 1) * sizeof(double)));
    double* bufs[2] = {base.ops.pool.d(), ops.pool.d()};
    TRY(lb.run(*this, bufs));
    return DMRG_OK;
}

// ====================================================== renormalisation
// New stored block from an enlarged block: kept merged sectors keep_m with
// kdim states; U (iso, comp_dim x k per kept sector) must already be in out.iso.
// O'[x', x] = U_{x'}^T O[x', x] U_x summed over the sub-sector blocks.
dmrg_status Engine::renormalize(const Enl& en, const OpSet& ops, bool normal_in, Stored& out,
                                const std::vector<int>& keep_m, const std::vector<int>& kdim) {
    std::vector<int> newidx(en.mq.size(), -1);
    for (size_t x = 0; x < keep_m.size(); ++x) newidx[keep_m[x]] = (int)x;
    // transition from normal to complementary pair operators?
    bool need_normal = out.side == 'L' ? left_normal(out.length()) : right_normal(out.lo);
    bool transition = normal_in && !need_normal;
    out.normal = normal_in && need_normal;
    OpSet tmp;   // renormalised A, B at the transition
    GB g1, g2;
    int64_t t_elems = 0;
    struct Pending {
        int which;   // 0 = out.ops, 1 = tmp
        Key key;
        Op op;
    };
    std::vector<Pending> pend;
    // per operator, its blocks grouped by (m_out, m_in) and within a group by
    // output sub-sector: formed on several host threads, then planned in
    // operator order below (pool offsets and plans are those of a serial pass)
    typedef std::vector<std::pair<int, std::vector<const Blk*>>> ByOut;
    struct OpGroups {
        std::vector<std::pair<std::pair<int, int>, ByOut>> groups;
    };
    std::vector<OpGroups> og(ops.ops.size());
    auto group_op = [&](size_t o) {
        std::map<std::pair<int, int>, std::map<int, std::vector<const Blk*>>> groups;
        for (const Blk& b : ops.ops[o].blk) {
            int mo = en.sub[b.out].m, mi = en.sub[b.in].m;
            if (newidx[mo] < 0 || newidx[mi] < 0) continue;
            groups[{mo, mi}][b.out].push_back(&b);
        }
        for (auto& gkv : groups) og[o].groups.push_back({gkv.first, ByOut(gkv.second.begin(), gkv.second.end())});
    };
    {
        std::atomic<size_t> next(0);
        auto run = [&] {
            for (size_t o = next++; o < ops.ops.size(); o = next++) group_op(o);
        };
        const int nth = host_threads((int64_t)ops.ops.size());
        std::vector<std::thread> pool;
        for (int t = 1; t < nth; ++t) pool.emplace_back(run);
        run();
        for (auto& th : pool) th.join();
    }
    for (size_t o = 0; o < ops.ops.size(); ++o) {
        const Key& key = ops.keys[o];
        const Op& op = ops.ops[o];
        bool to_tmp = transition && (key.k == 'A' || key.k == 'B');
        OpSet& dst = to_tmp ? tmp : out.ops;
        if (og[o].groups.empty()) continue;
        Op nop;
        nop.dq = op.dq;
        nop.par = op.par;
        for (auto& gkv : og[o].groups) {
            int mo = gkv.first.first, mi = gkv.first.second;
            int xo = newidx[mo], xi = newidx[mi];
            int ko = kdim[xo], ki = kdim[xi];
            Blk nb{xo, xi, dst.alloc_block(ko, ki), ko, ki};
            // phase 1: T[(i_out)] = sum_{i_in} O[i_out, i_in] U_mi[rows i_in]  (d(i_out) x ki)
            const ByOut& by_out = gkv.second;
            g2.begin();
            for (auto& bo : by_out) {
                const Sub& so = en.sub[bo.first];
                int64_t toff = t_elems;
                t_elems += ((int64_t)so.dim * ki + 31) / 32 * 32;
                g1.begin();
                for (const Blk* b : bo.second) {
                    const Sub& si = en.sub[b->in];
                    g1.chunk(1.0, 0, b->off, b->cols, false, 1, out.iso_off[xi] + (int64_t)si.off * ki, ki,
                             false, si.dim);
                }
                g1.end(2, toff, ki, so.dim, ki, 0);
                // phase 2 chunk: U_mo[rows i_out]^T T
                g2.chunk(1.0, 1, out.iso_off[xo] + (int64_t)so.off * ko, ko, true, 2, toff, ki, false, so.dim);
            }
            g2.end(to_tmp ? 4 : 3, nb.off, ki, ko, ki, 0);
            nop.blk.push_back(nb);
        }
        nop.index();
        pend.push_back({to_tmp ? 1 : 0, key, std::move(nop)});
    }
    for (auto& p : pend) (p.which ? tmp : out.ops).add(p.key, std::move(p.op));
    // device execution
    TRY(alloc_buf(out.ops.pool, std::max<int64_t>(out.ops.size, 1) * sizeof(double)));
    if (tmp.size) TRY(alloc_buf(tmp.pool, tmp.size * sizeof(double)));
    Buf tbuf;
    TRY(alloc_buf(tbuf, std::max<int64_t>(t_elems, 1) * sizeof(double)));
    GemmPlan p1, p2;
    TRY(finish_plans(*this, g1, p1, g2, p2));
    BufTable bufs{ops.pool.p, out.iso.p, tbuf.p, out.ops.pool.p, tmp.pool.p};
    TRY(run_gemm(dmrgdev::P_F64, bufs, p1));
    TRY(run_gemm(dmrgdev::P_F64, bufs, p2));
    if (!transition) return DMRG_OK;
    // complementary operators of the new block from its renormalised normal ones
    FormulaCtx F{*this, out};
    struct Item {
        Key key;
        Lin lin;
    };
    std::vector<Item> items;
    // helper view: resolve refs against tmp
    auto addk = [&](Lin& l, const Key& k, double c, bool tr) {
        if (c == 0.0) return;
        int x = tmp.find(k);
        if (x >= 0) l.refs.push_back({x, tr, c});
    };
    if (out.side == 'L') {
        for (int k = out.hi; k < N_; ++k)
            for (int l = k + 1; l < N_; ++l) {
                Lin lin;
                for (int i = out.lo; i < out.hi; ++i)
                    for (int j = i + 1; j < out.hi; ++j) addk(lin, {'A', i, j}, V(i, j, k, l), false);
                items.push_back({{'P', k, l}, lin});
            }
        for (int j = out.hi; j < N_; ++j)
            for (int l = j; l < N_; ++l) {
                Lin lin;
                for (int i = out.lo; i < out.hi; ++i)
                    for (int k = out.lo; k < out.hi; ++k) {
                        if (i <= k) addk(lin, {'B', i, k}, V(i, j, k, l), false);
                        else addk(lin, {'B', k, i}, V(i, j, k, l), true);
                    }
                items.push_back({{'Q', j, l}, lin});
            }
    } else {
        for (int i = 0; i < out.lo; ++i)
            for (int j = i + 1; j < out.lo; ++j) {
                Lin lin;
                for (int k = out.lo; k < out.hi; ++k)
                    for (int l = k + 1; l < out.hi; ++l) addk(lin, {'A', k, l}, V(i, j, k, l), true);
                items.push_back({{'P', i, j}, lin});
            }
        for (int i = 0; i < out.lo; ++i)
            for (int k = i; k < out.lo; ++k) {
                Lin lin;
                for (int j = out.lo; j < out.hi; ++j)
                    for (int l = out.lo; l < out.hi; ++l) {
                        if (j <= l) addk(lin, {'B', j, l}, V(i, j, k, l), false);
                        else addk(lin, {'B', l, j}, V(i, j, k, l), true);
                    }
                items.push_back({{'Q', i, k}, lin});
            }
    }
    (void)F;
    // new pool = old pool content + complementary ops
    OpSet comp;
    LB lb;
    std::vector<std::pair<Key, Op>> newops;
    for (auto& it : items) {
        if (it.lin.refs.empty()) continue;
        std::map<int, std::vector<LcTerm>> by_in;   // input sector -> terms
        std::map<int, int> out_of;
        QN dq;
        int par = 0;
        bool first = true;
        for (const Ref& r : it.lin.refs) {
            const Op& o = tmp.ops[r.op];
            QN odq = r.trans ? -o.dq : o.dq;
            if (first) {
                dq = odq;
                par = o.par;
                first = false;
            }
            for (const Blk& b : o.blk) {
                int in = r.trans ? b.out : b.in, ot = r.trans ? b.in : b.out;
                LcTerm lt{};
                lt.coef = r.coef;
                lt.src_off = b.off;
                lt.ld = b.cols;
                lt.trans = r.trans;
                lt.buf = 0;
                by_in[in].push_back(lt);
                out_of[in] = ot;
            }
        }
        Op op;
        op.dq = dq;
        op.par = par;
        for (auto& kv : by_in) {
            int in = kv.first, ot = out_of[in];
            Blk nb{ot, in, out.ops.size + comp.alloc_block(kdim[ot], kdim[in]), kdim[ot], kdim[in]};
            op.blk.push_back(nb);
            lb.block(1, nb.off - out.ops.size, nb.rows, nb.cols, kv.second);
        }
        op.index();
        newops.push_back({it.key, std::move(op)});
    }
    // grow the pool: copy the renormalised part, then the combinations
    Buf np;
    TRY(alloc_buf(np, std::max<int64_t>(out.ops.size + comp.size, 1) * sizeof(double)));
    DEV(dmrgdev::d2d(dev_, np.p, out.ops.pool.p, out.ops.size * sizeof(double)));
    double* bufs2[2] = {tmp.pool.d(), np.d() + out.ops.size};
    TRY(lb.run(*this, bufs2));
    out.ops.size += comp.size;
    out.ops.pool = std::move(np);
    for (auto& kv : newops) out.ops.add(kv.first, std::move(kv.second));
    return DMRG_OK;
}

// =============================================================== bonds
dmrg_status Engine::setup_bond(int b, std::unique_ptr<Bond>& outp) {
    double t0 = now();
    auto B = std::make_unique<Bond>();
    B->b = b;
    B->gen = ++bond_gen_;
    const Stored& L = *L_[b];
    const Stored& R = *R_[b + 2];
    // E sectors: complementable by the sites 0..b
    std::vector<QN> eq;
    {
        std::set<QN> cand;
        for (int sg = 0; sg < 2; ++sg)
            for (const QN& q : R.basis.q) cand.insert(sg ? q + delta_[b + 1] : q);
        for (const QN& q : cand)
            if (reachable(pre_[b + 1], T_ - q)) eq.push_back(q);
    }
    // S sectors: partner in E; then E sectors: partner in S
    std::vector<QN> sq;
    {
        std::set<QN> es(eq.begin(), eq.end()), cand;
        for (int sg = 0; sg < 2; ++sg)
            for (const QN& q : L.basis.q) cand.insert(sg ? q + delta_[b] : q);
        for (const QN& q : cand)
            if (es.count(T_ - q)) sq.push_back(q);
        std::set<QN> ss(sq.begin(), sq.end());
        std::vector<QN> eq2;
        for (const QN& q : eq)
            if (ss.count(T_ - q)) eq2.push_back(q);
        eq.swap(eq2);
    }
    // plan the two enlarged blocks on two host threads, then queue their copies
    {
        LB lbL, lbR;
        std::string whyL, whyR;
        bool okL = false, okR = false;
        std::thread tl([&] { okL = enlarge_plan(L, 'L', sq, B->S, B->Sops, lbL, whyL); });
        okR = enlarge_plan(R, 'R', eq, B->E, B->Eops, lbR, whyR);
        tl.join();
        if (!okL) return fail(DMRG_ERR_DEVICE, whyL);
        if (!okR) return fail(DMRG_ERR_DEVICE, whyR);
        TRY(enlarge_run(L, B->Sops, lbL));
        TRY(enlarge_run(R, B->Eops, lbR));
    }
    // psi layout: merged S sectors in order
    B->blk_of_S.assign(B->S.mq.size(), -1);
    for (size_t m = 0; m < B->S.mq.size(); ++m) {
        int me = B->E.find_m(T_ - B->S.mq[m]);
        if (me < 0) continue;
        B->blk_of_S[m] = (int)B->pm_S.size();
        B->pm_S.push_back((int)m);
        B->pm_E.push_back(me);
        B->poff.push_back(B->dim);
        B->dim += (int64_t)B->S.md[m] * B->E.md[me];
    }
    // H_eff terms of the S|E split of H: H_S, H_E; pair terms with the two-body sums
    // carried by complementary operators of the larger side; the 3+1 and 1+3 terms
    auto& T = B->terms;
    const OpSet &So = B->Sops, &Eo = B->Eops;
    T.push_back({1.0, So.find({'H', 0, 0}), -1, false, false, false, 0});
    T.push_back({1.0, -1, Eo.find({'H', 0, 0}), false, false, false, 0});
    auto pair = [&](const Key& ka, bool ta, const Key& kb, bool tb, int par, bool hc) {
        int a = So.find(ka), c = Eo.find(kb);
        if (a < 0 || c < 0) return;
        T.push_back({1.0, a, c, ta, tb, false, par});
        if (hc) T.push_back({1.0, a, c, !ta, !tb, true, par});
    };
    if (normal_S(b)) {
        for (int i = 0; i <= b; ++i) {
            for (int j = i + 1; j <= b; ++j) pair({'A', i, j}, false, {'P', i, j}, false, 0, true);
            for (int k = i; k <= b; ++k) pair({'B', i, k}, false, {'Q', i, k}, false, 0, i < k);
        }
    } else {
        for (int k = b + 1; k < N_; ++k) {
            for (int l = k + 1; l < N_; ++l) pair({'P', k, l}, false, {'A', k, l}, true, 0, true);
            for (int l = k; l < N_; ++l) pair({'Q', k, l}, false, {'B', k, l}, false, 0, k < l);
        }
    }
    for (int l = b + 1; l < N_; ++l) pair({'R', l, 0}, false, {'C', l, 0}, true, 1, true);
    for (int i = 0; i <= b; ++i) pair({'C', i, 0}, false, {'R', i, 0}, false, 1, true);
    TRY(build_heff_plan(*B));
    TRY(build_diag(*B));
    acc_.blocking_seconds += now() - t0;
    outp = std::move(B);
    return DMRG_OK;
}

// Launches per product: phase 1 forms Z_t[x, i] = psi_x[i, :] op(B_t)^T for
// every term t with an E operator, one row block per input S sub-sector i,
// spanning the full width of the output E sector (its sub-sectors side by
// side; columns a term does not reach are cleared).  Phase 2 then gives
// every output row block Y[x2, i2, :] (full E width) all of its terms as one
// stacked-K chunk list: sum_t alpha op(A_t)[i2 <- i] Z_t[x, i] (or op(A) psi
// for the S-only term).  The E-only term (1 x H_E) is a third, small launch
// that accumulates psi op(B)^T into the sub-blocks.  Terms are grouped so
// that each group's Z fits the scratch budget; the first group writes every
// output block, later groups accumulate.
// bufs: 0 S ops, 1 E ops, 2 x, 3 Z, 4 y.
dmrg_status Engine::build_heff_plan(Bond& B) {
    const Enl &S = B.S, &E = B.E;
    const int nb = (int)B.pm_S.size();
    auto yid = [&](int x, int i2) { return x * 2 + S.sub[i2].sigma; };
    auto subid = [&](int x, int i, int j) { return x * 4 + S.sub[i].sigma * 2 + E.sub[j].sigma; };
    const int64_t zbudget =
        opt_.scratch_bytes ? (int64_t)(opt_.scratch_bytes / sizeof(double)) : ((int64_t)1 << 31);
    std::vector<std::pair<int, int>> rows(nb * 2, {-1, -1});   // yid -> (x, i2)
    for (int x = 0; x < nb; ++x)
        for (int i : S.msub[B.pm_S[x]])
            if (i >= 0) rows[yid(x, i)] = {x, i};

    // one Z output block (a sub-sector's columns of a term's Z row block)
    struct ZOut {
        int64_t zoff;   // relative to the term's own Z
        int ldz, M, N;
        std::vector<GemmChunk> chunks;
    };
    struct TermWork {
        std::vector<ZOut> z;
        std::vector<std::pair<int, GemmChunk>> c2;   // (yid, chunk); Z offsets relative
        std::vector<int> n2;                         // per c2 chunk: columns that can be nonzero
        std::vector<std::pair<int, GemmChunk>> c3;   // (subid, chunk) of the E-only term
        int64_t zsize = 0;
        double alg = 0.0;                            // algorithmic flops
    };
    // (work runs on several host threads: it reports, the caller fails)
    auto leaves = [&]() { return DMRG_ERR_DEVICE; };
    auto work = [&](const Term& tm, TermWork& w) -> dmrg_status {
        const Op* A = tm.a >= 0 ? &B.Sops.ops[tm.a] : nullptr;
        const Op* Bo = tm.b >= 0 ? &B.Eops.ops[tm.b] : nullptr;
        auto alpha_of = [&](int i, int i2) {
            double sg = 1.0;
            if (tm.par) sg = ((tm.sign_out ? S.sub[i2].q.n() : S.sub[i].q.n()) & 1) ? -1.0 : 1.0;
            return tm.coef * sg;
        };
        for (int x = 0; x < nb; ++x) {
            const int mS = B.pm_S[x], mE = B.pm_E[x];
            const int ldx = E.md[mE];
            // Algorithmic flops of the term on this block: the cheaper of the two
            // contraction orders, over the nonzero sub-sector blocks (A: i -> i2,
            // B: j -> j2) with each intermediate formed once:
            //   B first: 2 (sum_{i acted on} d_i) sum_B d_j d_j2 + 2 sum_A d_i d_i2 (sum_{j2 reached} d_j2)
            //   A first: 2 sum_A d_i d_i2 (sum_{j acted on} d_j) + 2 (sum_{i2 reached} d_i2) sum_B d_j d_j2
            {
                double sa = 0.0, sb = 0.0, din = 0.0, dout = 0.0, ein = 0.0, eout = 0.0;
                if (A) {
                    std::set<int> i_out;
                    for (int i : S.msub[mS]) {
                        if (i < 0 || A->acting(i, tm.ta).empty()) continue;
                        din += S.sub[i].dim;
                        for (int ai : A->acting(i, tm.ta)) {
                            const int i2 = tm.ta ? A->blk[ai].in : A->blk[ai].out;
                            sa += (double)S.sub[i].dim * S.sub[i2].dim;
                            i_out.insert(i2);
                        }
                    }
                    for (int i2 : i_out) dout += S.sub[i2].dim;
                }
                if (Bo) {
                    std::set<int> j_out;
                    for (int j : E.msub[mE]) {
                        if (j < 0 || Bo->acting(j, tm.tb).empty()) continue;
                        ein += E.sub[j].dim;
                        for (int bi : Bo->acting(j, tm.tb)) {
                            const int j2 = tm.tb ? Bo->blk[bi].in : Bo->blk[bi].out;
                            sb += (double)E.sub[j].dim * E.sub[j2].dim;
                            j_out.insert(j2);
                        }
                    }
                    for (int j2 : j_out) eout += E.sub[j2].dim;
                }
                if (A && Bo) w.alg += 2.0 * std::min(din * sb + sa * eout, sa * ein + dout * sb);
                else if (A) w.alg += 2.0 * sa * ldx;
                else if (Bo) w.alg += 2.0 * S.md[mS] * sb;
            }
            // When the S operator acts on every sub-sector of this block, Z_t for
            // the whole block (all its rows) is formed at once: taller phase-1
            // output blocks, one operator read per block row tile.
            bool zrow_done = false;
            int64_t zrow = 0;
            int NE2x = 0, NE2use = 0;
            if (A && Bo) {
                bool all = true;
                for (int i : S.msub[mS])
                    if (i >= 0 && A->acting(i, tm.ta).empty()) all = false;
                std::vector<std::pair<int, int>> fd[2];
                int m2 = -1;
                for (int j : E.msub[mE]) {
                    if (j < 0) continue;
                    for (int bi : Bo->acting(j, tm.tb)) {
                        const Blk& bb = Bo->blk[bi];
                        const int j2 = tm.tb ? bb.in : bb.out;
                        if (m2 >= 0 && E.sub[j2].m != m2) return leaves();
                        m2 = E.sub[j2].m;
                        fd[E.sub[j2].sigma].push_back({j, bi});
                    }
                }
                if (all && m2 >= 0) {
                    NE2x = E.md[m2];
                    NE2use = 0;
                    for (int j2 : E.msub[m2])
                        if (j2 >= 0 && !fd[E.sub[j2].sigma].empty()) NE2use += E.sub[j2].dim;
                    const int dS = S.md[mS];
                    zrow = w.zsize;
                    w.zsize += ((int64_t)dS * NE2x + 7) / 8 * 8;
                    for (int j2 : E.msub[m2]) {
                        if (j2 < 0) continue;
                        ZOut out;
                        out.zoff = zrow + E.sub[j2].off;
                        out.ldz = NE2x;
                        out.M = dS;
                        out.N = E.sub[j2].dim;
                        for (auto& f : fd[E.sub[j2].sigma]) {
                            const Blk& bb = Bo->blk[f.second];
                            const int j = f.first;
                            out.chunks.push_back(GemmChunk{1.0, B.poff[x] + E.sub[j].off, bb.off, ldx, bb.cols,
                                                           E.sub[j].dim, 2, 1, 0, (uint8_t)!tm.tb});
                        }
                        w.z.push_back(std::move(out));
                    }
                    zrow_done = true;
                }
            }
            for (int i : S.msub[mS]) {
                if (i < 0) continue;
                const int di = S.sub[i].dim;
                const int64_t xrow = B.poff[x] + (int64_t)S.sub[i].off * ldx;
                if (!Bo) {   // S-only term: op(A) psi over the full width
                    if (!A) continue;
                    for (int ai : A->acting(i, tm.ta)) {
                        const Blk& ab = A->blk[ai];
                        const int i2 = tm.ta ? ab.in : ab.out;
                        const int x2 = B.blk_of_S[S.sub[i2].m];
                        if (x2 < 0 || B.pm_E[x2] != mE) return leaves();
                        w.c2.push_back({yid(x2, i2), GemmChunk{alpha_of(i, i2), ab.off, xrow, ab.cols, ldx, di, 0, 2,
                                                               (uint8_t)tm.ta, 0}});
                        w.n2.push_back(ldx);
                    }
                    continue;
                }
                // no S block on this sub-sector: no Z row block is needed
                if (A && A->acting(i, tm.ta).empty()) continue;
                // E operator: which input sub-sectors j feed which output sub-sector j2
                std::vector<std::pair<int, int>> feeds[2];   // per output sigma: (j, block)
                int mE2 = -1;
                for (int j : E.msub[mE]) {
                    if (j < 0) continue;
                    for (int bi : Bo->acting(j, tm.tb)) {
                        const Blk& bb = Bo->blk[bi];
                        const int j2 = tm.tb ? bb.in : bb.out;
                        if (mE2 >= 0 && E.sub[j2].m != mE2) return leaves();
                        mE2 = E.sub[j2].m;
                        feeds[E.sub[j2].sigma].push_back({j, bi});
                    }
                }
                if (mE2 < 0) continue;
                if (!A) {   // E-only term: psi op(B)^T into the sub-blocks (third launch)
                    const int x2 = B.blk_of_S[S.sub[i].m];
                    if (x2 < 0 || B.pm_E[x2] != mE2) return leaves();
                    for (int sg = 0; sg < 2; ++sg)
                        for (auto& f : feeds[sg]) {
                            const Blk& bb = Bo->blk[f.second];
                            const int j = f.first, j2 = tm.tb ? bb.in : bb.out;
                            w.c3.push_back({subid(x2, i, j2),
                                            GemmChunk{alpha_of(i, i), xrow + E.sub[j].off, bb.off, ldx, bb.cols,
                                                      E.sub[j].dim, 2, 1, 0, (uint8_t)!tm.tb}});
                        }
                    continue;
                }
                // Z_t[x, i]: d_i x NE2, sub-sector j2 at its column offset (rows of
                // several i of one block are contiguous when they share a Z, below)
                int64_t zo;
                if (zrow_done) {
                    zo = zrow + (int64_t)S.sub[i].off * NE2x;
                } else {
                    zo = w.zsize;
                    w.zsize += ((int64_t)di * E.md[mE2] + 7) / 8 * 8;
                }
                const int NE2 = E.md[mE2];
                int use = NE2x ? NE2use : 0;
                if (!zrow_done) {
                    use = 0;
                    for (int j2 : E.msub[mE2])
                        if (j2 >= 0 && !feeds[E.sub[j2].sigma].empty()) use += E.sub[j2].dim;
                    for (int j2 : E.msub[mE2]) {
                        if (j2 < 0) continue;
                        ZOut out;
                        out.zoff = zo + E.sub[j2].off;
                        out.ldz = NE2;
                        out.M = di;
                        out.N = E.sub[j2].dim;
                        for (auto& f : feeds[E.sub[j2].sigma]) {
                            const Blk& bb = Bo->blk[f.second];
                            const int j = f.first;
                            out.chunks.push_back(GemmChunk{1.0, xrow + E.sub[j].off, bb.off, ldx, bb.cols,
                                                           E.sub[j].dim, 2, 1, 0, (uint8_t)!tm.tb});
                        }
                        w.z.push_back(std::move(out));   // no chunks: the columns are cleared
                    }
                }
                for (int ai : A->acting(i, tm.ta)) {
                    const Blk& ab = A->blk[ai];
                    const int i2 = tm.ta ? ab.in : ab.out;
                    const int x2 = B.blk_of_S[S.sub[i2].m];
                    if (x2 < 0 || B.pm_E[x2] != mE2) return leaves();
                    w.c2.push_back(
                        {yid(x2, i2), GemmChunk{alpha_of(i, i2), ab.off, zo, ab.cols, NE2, di, 0, 3, (uint8_t)tm.ta, 0}});
                    w.n2.push_back(use);
                }
            }
        }
        return DMRG_OK;
    };

    B.groups.clear();
    B.flops = 0.0;
    B.flops_alg = 0.0;
    std::vector<std::vector<GemmChunk>> lists(nb * 2), lists3(nb * 4);
    std::vector<std::vector<int>> lists_n(nb * 2);
    GB g1;
    int64_t z = 0;
    bool first = true;
    auto close_group = [&]() -> dmrg_status {
        HeffGroup grp;
        grp.z_elems = z;
        GB g2, g3;
        for (int id = 0; id < nb * 2; ++id) {
            const int x = rows[id].first, i2 = rows[id].second;
            if (x < 0) continue;
            auto& l = lists[id];
            if (!first && l.empty()) continue;
            g2.begin();
            g2.chunks.insert(g2.chunks.end(), l.begin(), l.end());
            g2.nuse.insert(g2.nuse.end(), lists_n[id].begin(), lists_n[id].end());
            const int ldy = E.md[B.pm_E[x]];
            g2.end(4, B.poff[x] + (int64_t)S.sub[i2].off * ldy, ldy, S.sub[i2].dim, ldy, first ? 0 : 1);
            l.clear();
            lists_n[id].clear();
        }
        for (int id = 0; id < nb * 4; ++id) {
            auto& l = lists3[id];
            if (l.empty()) continue;
            const int x = id / 4;
            int i = -1, j = -1;
            for (int ii : S.msub[B.pm_S[x]])
                if (ii >= 0 && S.sub[ii].sigma == (id & 3) / 2) i = ii;
            for (int jj : E.msub[B.pm_E[x]])
                if (jj >= 0 && E.sub[jj].sigma == (id & 1)) j = jj;
            if (i < 0 || j < 0) return fail(DMRG_ERR_DEVICE, "internal: E-only term without its sub-block");
            g3.begin();
            g3.chunks.insert(g3.chunks.end(), l.begin(), l.end());
            const int ldy = E.md[B.pm_E[x]];
            g3.end(4, B.poff[x] + (int64_t)S.sub[i].off * ldy + E.sub[j].off, ldy, S.sub[i].dim, E.sub[j].dim, 1);
            l.clear();
        }
        TRY(finish_plans(*this, g1, grp.p1, g2, grp.p2));
        TRY(finish_plan(*this, g3, grp.p3));
        B.flops += grp.p1.flops + grp.p2.flops + grp.p3.flops;
        B.groups.push_back(std::move(grp));
        g1 = GB();
        z = 0;
        first = false;
        return DMRG_OK;
    };
    // Every term's blocks and chunks depend only on the bond's structure: they
    // are formed on up to 16 host threads, then merged in term order (the
    // plans are those of a serial pass).
    const size_t nterms = B.terms.size();
    std::vector<TermWork> works(nterms);
    {
        std::vector<dmrg_status> wst(nterms, DMRG_OK);
        std::atomic<size_t> next(0);
        auto run = [&] {
            for (size_t t = next++; t < nterms; t = next++) wst[t] = work(B.terms[t], works[t]);
        };
        const int nth = host_threads((int64_t)nterms);
        std::vector<std::thread> pool;
        for (int i = 1; i < nth; ++i) pool.emplace_back(run);
        run();
        for (auto& th : pool) th.join();
        for (dmrg_status st : wst)
            if (st != DMRG_OK) return fail(DMRG_ERR_DEVICE, "internal: H_eff term leaves the target sector");
    }
    for (size_t t = 0; t < nterms; ++t) {
        TermWork w = std::move(works[t]);
        if (z > 0 && z + w.zsize > zbudget) TRY(close_group());
        for (ZOut& zb : w.z) {
            g1.begin();
            g1.chunks.insert(g1.chunks.end(), zb.chunks.begin(), zb.chunks.end());
            g1.end(3, z + zb.zoff, zb.ldz, zb.M, zb.N, 0);
        }
        for (size_t q = 0; q < w.c2.size(); ++q) {
            GemmChunk c = w.c2[q].second;
            if (c.b_buf == 3) c.b_off += z;
            lists[w.c2[q].first].push_back(c);
            lists_n[w.c2[q].first].push_back(w.n2[q]);
        }
        B.flops_alg += w.alg;
        for (auto& pc : w.c3) lists3[pc.first].push_back(pc.second);
        z += w.zsize;
    }
    TRY(close_group());
    int64_t zmax = 0;
    for (auto& g : B.groups) zmax = std::max(zmax, g.z_elems);
    if ((int64_t)(z_.bytes / sizeof(double)) < zmax)
        TRY(alloc_buf(z_, std::max<int64_t>(zmax, 1) * sizeof(double)));
    return DMRG_OK;
}

dmrg_status Engine::build_diag(Bond& B) {
    const Enl &S = B.S, &E = B.E;
    std::vector<DiagTask> tasks;
    std::vector<DiagTerm> terms;
    for (size_t x = 0; x < B.pm_S.size(); ++x) {
        int mS = B.pm_S[x], mE = B.pm_E[x];
        int ld = E.md[mE];
        for (int i : S.msub[mS]) {
            if (i < 0) continue;
            for (int j : E.msub[mE]) {
                if (j < 0) continue;
                int32_t t0 = (int32_t)terms.size();
                for (const Term& tm : B.terms) {
                    const Op* A = tm.a >= 0 ? &B.Sops.ops[tm.a] : nullptr;
                    const Op* Bo = tm.b >= 0 ? &B.Eops.ops[tm.b] : nullptr;
                    if ((A && A->dq != QN()) || (Bo && Bo->dq != QN())) continue;
                    DiagTerm d{};
                    d.coef = tm.coef;
                    const Blk* ab = nullptr;
                    const Blk* bb = nullptr;
                    if (A)
                        for (int q : A->ins(i))
                            if (A->blk[q].out == i) ab = &A->blk[q];
                    if (Bo)
                        for (int q : Bo->ins(j))
                            if (Bo->blk[q].out == j) bb = &Bo->blk[q];
                    if (A) {
                        if (!ab) continue;
                        d.a_off = ab->off;
                        d.a_step = ab->cols + 1;
                        d.a_buf = 0;
                    } else {
                        d.a_ident = 1;
                    }
                    if (Bo) {
                        if (!bb) continue;
                        d.b_off = bb->off;
                        d.b_step = bb->cols + 1;
                        d.b_buf = 1;
                    } else {
                        d.b_ident = 1;
                    }
                    terms.push_back(d);
                }
                int32_t t1 = (int32_t)terms.size();
                int rows = S.sub[i].dim, cols = E.sub[j].dim;
                int64_t off = B.poff[x] + (int64_t)S.sub[i].off * ld + E.sub[j].off;
                for (int r0 = 0; r0 < rows; r0 += 32)
                    for (int c0 = 0; c0 < cols; c0 += 32)
                        tasks.push_back({off, ld, r0, c0, std::min(32, rows - r0), std::min(32, cols - c0), t0, t1});
            }
        }
    }
    TRY(alloc_buf(B.diag, std::max<int64_t>(B.dim, 1) * sizeof(double)));
    Buf dt, dterm;
    TRY(upload(dt, tasks));
    TRY(upload(dterm, terms));
    double* bufs[3] = {B.Sops.pool.d(), B.Eops.pool.d(), B.diag.d()};
    if (!tasks.empty()) DEV(dmrgdev::diag(dev_, bufs, dt.as<DiagTask>(), (int)tasks.size(), dterm.as<DiagTerm>()));
    return DMRG_OK;
}

dmrg_status Engine::ensure_lo(Bond& B, int prec) {
    if (B.lo_prec == prec) return DMRG_OK;
    for (OpSet* o : {&B.Sops, &B.Eops}) {
        size_t es = prec == dmrgdev::P_F32 ? 4 : 2;
        TRY(alloc_buf(o->pool_lo, std::max<int64_t>(o->size, 1) * es));
        DEV(dmrgdev::convert(dev_, dmrgdev::P_F64, o->pool.p, prec, o->pool_lo.p, o->size));
        o->lo_prec = prec;
    }
    B.lo_prec = prec;
    return DMRG_OK;
}

// y = H_eff x (device pointers, FP64 I/O)
dmrg_status Engine::heff(Bond& B, const double* x, double* y, int prec) {
    DEV(dmrgdev::event_record(dev_, 0));
    TRY(heff_launch(B, x, y, prec, true));
    DEV(dmrgdev::event_record(dev_, 1));
    heff_time_ += dmrgdev::event_elapsed(dev_, 0, 1);
    return DMRG_OK;
}

// one product with per-phase event timing (the events add no synchronisation;
// the elapsed times are read after the product completes)
dmrg_status Engine::heff_launch(Bond& B, const double* x, double* y, int prec, bool timed) {
    if (batch_ && B.groups.size() == 1) return heff_batched(B, x, y, prec);
    if (opt_.graph && !in_many_ && B.groups.size() == 1) return heff_graph(B, x, y, prec);
    return heff_direct(B, x, y, prec, timed);
}

// The bond's product as a HIP graph: captured at the bond's first product in
// this precision, after every buffer it touches has its final size (nothing
// is allocated or synchronised during the capture), and replayed for later
// products; x and y pass through fixed staging vectors.
dmrg_status Engine::heff_graph(Bond& B, const double* x, double* y, int prec) {
    if (graph_exec_ && (graph_gen_ != B.gen || graph_prec_ != prec)) {
        dmrgdev::graph_destroy(graph_exec_);
        graph_exec_ = nullptr;
    }
    if (!graph_exec_) {
        const size_t vb = (size_t)std::max<int64_t>(B.dim, 1) * sizeof(double);
        if (gin_.bytes < vb) TRY(alloc_buf(gin_, vb));
        if (gout_.bytes < vb) TRY(alloc_buf(gout_, vb));
        const HeffGroup& g = B.groups[0];
        if (prec != dmrgdev::P_F64) {
            TRY(ensure_lo(B, prec));
            const size_t esz = prec == dmrgdev::P_F32 ? 4 : 2;
            if (xlo_.bytes < (size_t)B.dim * esz) TRY(alloc_buf(xlo_, std::max<int64_t>(B.dim, 1) * esz));
            if (ylo_.bytes < (size_t)B.dim * 4) TRY(alloc_buf(ylo_, std::max<int64_t>(B.dim, 1) * 4));
            const size_t zbytes = (size_t)std::max<int64_t>(g.z_elems, 1) * esz;
            if (scr_a_.bytes < zbytes) TRY(alloc_buf(scr_a_, zbytes));
        }
        const int64_t slots = std::max({g.p1.nslots, g.p2.nslots, g.p3.nslots});
        if (slots) TRY(ensure_partials(slots));
        DEV(dmrgdev::graph_begin(dev_));
        dmrg_status st = heff_direct(B, gin_.d(), gout_.d(), prec, false);
        void* ex = nullptr;
        const int rc = dmrgdev::graph_end(dev_, &ex);
        if (st < 0) {
            dmrgdev::graph_destroy(ex);
            return st;
        }
        if (rc) return fail(DMRG_ERR_DEVICE, dmrgdev::last_error(dev_));
        graph_exec_ = ex;
        graph_gen_ = B.gen;
        graph_prec_ = prec;
    }
    DEV(dmrgdev::d2d(dev_, gin_.p, x, (size_t)B.dim * sizeof(double)));
    DEV(dmrgdev::graph_launch(dev_, graph_exec_));
    DEV(dmrgdev::d2d(dev_, y, gout_.p, (size_t)B.dim * sizeof(double)));
    return DMRG_OK;
}

dmrg_status Engine::heff_direct(Bond& B, const double* x, double* y, int prec, bool timed) {
    const double es = prec == dmrgdev::P_F64 ? 8.0 : (prec == dmrgdev::P_F32 ? 4.0 : 2.0);
    if (prec == dmrgdev::P_F64) {
        for (size_t g = 0; g < B.groups.size(); ++g) {
            BufTable bufs{B.Sops.pool.p, B.Eops.pool.p, (void*)x, z_.p, y};
            TRY(run_gemm(prec, bufs, B.groups[g].p1, -1, dmrgdev::GK_HEFF_Z, nullptr, timed ? 2 : -1, timed ? 3 : -1));
            TRY(run_gemm(prec, bufs, B.groups[g].p2, -1, dmrgdev::GK_HEFF_Y, nullptr, timed ? 6 : -1, timed ? 4 : -1));
            if (timed) DEV(dmrgdev::event_record(dev_, 5));
            TRY(run_gemm(prec, bufs, B.groups[g].p3));
            if (timed && opt_.precision == DMRG_FP64) account(B.groups[g], es, es);
        }
        return DMRG_OK;
    }
    TRY(ensure_lo(B, prec));
    const size_t esz = prec == dmrgdev::P_F32 ? 4 : 2;
    int64_t zmax = 0;
    for (auto& g : B.groups) zmax = std::max(zmax, g.z_elems);
    if (xlo_.bytes < (size_t)B.dim * esz) TRY(alloc_buf(xlo_, std::max<int64_t>(B.dim, 1) * esz));
    if (ylo_.bytes < (size_t)B.dim * 4) TRY(alloc_buf(ylo_, std::max<int64_t>(B.dim, 1) * 4));
    size_t zbytes = (size_t)std::max<int64_t>(zmax, 1) * esz;
    if (scr_a_.bytes < zbytes) TRY(alloc_buf(scr_a_, zbytes));
    DEV(dmrgdev::convert(dev_, dmrgdev::P_F64, x, prec, xlo_.p, B.dim));
    for (size_t g = 0; g < B.groups.size(); ++g) {
        BufTable bufs{B.Sops.pool_lo.p, B.Eops.pool_lo.p, xlo_.p, scr_a_.p, ylo_.p};
        // Z in the operand precision
        TRY(run_gemm(prec, bufs, B.groups[g].p1, prec, dmrgdev::GK_HEFF_Z, nullptr, timed ? 2 : -1, timed ? 3 : -1));
        TRY(run_gemm(prec, bufs, B.groups[g].p2, dmrgdev::P_F32, dmrgdev::GK_HEFF_Y, nullptr, timed ? 6 : -1,
                     timed ? 4 : -1));
        if (timed) DEV(dmrgdev::event_record(dev_, 5));
        TRY(run_gemm(prec, bufs, B.groups[g].p3, dmrgdev::P_F32));
        if (timed) account(B.groups[g], es, es);
    }
    DEV(dmrgdev::convert(dev_, dmrgdev::P_F32, ylo_.p, dmrgdev::P_F64, y, B.dim));
    return DMRG_OK;
}

// The product of heff_launch through the batch: the input conversion and the
// output conversion stay on the context stream; the three GEMM phases and
// their reductions are launched by the batch together with the products of
// the other contexts pending at the time (same plans, same buffers).
dmrg_status Engine::heff_batched(Bond& B, const double* x, double* y, int prec) {
    const HeffGroup& g = B.groups[0];
    BufTable bufs{};
    int cp1 = prec, cp2 = prec;
    const bool low = prec != dmrgdev::P_F64;
    if (!low) {
        bufs = BufTable{B.Sops.pool.p, B.Eops.pool.p, (void*)x, z_.p, y};
    } else {
        TRY(ensure_lo(B, prec));
        const size_t esz = prec == dmrgdev::P_F32 ? 4 : 2;
        if (xlo_.bytes < (size_t)B.dim * esz) TRY(alloc_buf(xlo_, std::max<int64_t>(B.dim, 1) * esz));
        if (ylo_.bytes < (size_t)B.dim * 4) TRY(alloc_buf(ylo_, std::max<int64_t>(B.dim, 1) * 4));
        const size_t zbytes = (size_t)std::max<int64_t>(g.z_elems, 1) * esz;
        if (scr_a_.bytes < zbytes) TRY(alloc_buf(scr_a_, zbytes));
        DEV(dmrgdev::convert(dev_, dmrgdev::P_F64, x, prec, xlo_.p, B.dim));
        bufs = BufTable{B.Sops.pool_lo.p, B.Eops.pool_lo.p, xlo_.p, scr_a_.p, ylo_.p};
        cp2 = dmrgdev::P_F32;
    }
    const int64_t slots = std::max({g.p1.nslots, g.p2.nslots, g.p3.nslots});
    if (slots) {
        TRY(ensure_partials(slots));
        bufs[dmrgdev::kPartialBuf] = partial_.p;
    }
    if (!ev_ready_) ev_ready_ = dmrgdev::xevent_create(dev_);
    if (!ev_done_) ev_done_ = dmrgdev::xevent_create(dev_);
    if (!ev_ready_ || !ev_done_) return fail(DMRG_ERR_DEVICE, dmrgdev::last_error(dev_));
    HeffRequest r;
    r.ab_prec = prec;
    r.c_prec[0] = cp1;
    r.c_prec[1] = r.c_prec[2] = cp2;
    const GemmPlan* ps[3] = {&g.p1, &g.p2, &g.p3};
    for (int ph = 0; ph < 3; ++ph) {
        const GemmPlan& p = *ps[ph];
        for (int i = 0; i < dmrgdev::kMaxBufs; ++i) r.plan[ph].bufs[i] = r.red[ph].bufs[i] = bufs[i];
        r.plan[ph].tasks = p.tasks;
        r.plan[ph].chunks = p.chunks;
        r.plan[ph].sc = dmrgdev::Sched{p.wg_off, std::max(1, p.nwg), p.nfull, p.ntasks};
        r.nwg[ph] = p.ntasks ? std::max(1, p.nwg) : 0;
        r.red[ph].reds = p.reds;
        r.nreds[ph] = p.nreds;
    }
    r.ready = ev_ready_;
    r.done = ev_done_;
    DEV(dmrgdev::xevent_record(dev_, ev_ready_));
    if (batch_->run(r)) return fail(DMRG_ERR_DEVICE, "grouped launch: " + batch_->error());
    DEV(dmrgdev::xevent_wait(dev_, ev_done_));
    if (low) DEV(dmrgdev::convert(dev_, dmrgdev::P_F32, ylo_.p, dmrgdev::P_F64, y, B.dim));
    return DMRG_OK;
}

void Engine::account(const HeffGroup& g, double es1, double es2) {
    // kernel intervals recorded by the launches themselves; the split-K
    // reduction runs between the end of phase 2 and event 5
    double t1 = dmrgdev::event_elapsed(dev_, 2, 3), t2 = dmrgdev::event_elapsed(dev_, 6, 4);
    acc_.reduce_seconds += dmrgdev::event_elapsed(dev_, 4, 5);
    if (g.p1.ntasks) {
        acc_.gemm1_launches += 1;
        acc_.gemm1_seconds += t1;
        acc_.gemm1_flops += g.p1.flops;
        acc_.gemm1_issued_flops += g.p1.issued;
        acc_.gemm1_bytes += g.p1.elems * es1;
    }
    if (g.p2.ntasks) {
        acc_.gemm2_launches += 1;
        acc_.gemm2_seconds += t2;
        acc_.gemm2_flops += g.p2.flops;
        acc_.gemm2_issued_flops += g.p2.issued;
        acc_.gemm2_bytes += g.p2.elems * es2;
    }
}

// =============================================================== Davidson
dmrg_status Engine::ensure_dv(int64_t n, int kmax) {
    if (dv_cap_ >= n && dv_V_.p) return DMRG_OK;
    int64_t cap = std::max<int64_t>(n, 1);
    TRY(alloc_buf(dv_V_, (size_t)cap * kmax * sizeof(double)));
    TRY(alloc_buf(dv_W_, (size_t)cap * kmax * sizeof(double)));
    TRY(alloc_buf(dv_x_, cap * sizeof(double)));
    TRY(alloc_buf(dv_hx_, cap * sizeof(double)));
    TRY(alloc_buf(dv_r_, cap * sizeof(double)));
    TRY(alloc_buf(dv_t_, cap * sizeof(double)));
    TRY(alloc_buf(dv_small_, 4096 * sizeof(double)));
    dv_cap_ = cap;
    return DMRG_OK;
}

// Lowest eigenpair of H_eff from the guess in psi_: subspace V from the
// normalised guess; correction r / (diag - theta) (|diag - theta| >= 1e-12);
// classical Gram-Schmidt twice; restart to [x] at the maximum subspace;
// converged when |H x - theta x| <= tol.
//
// Mixed modes (FP64 residual correction): expansion products run in reduced
// precision; the subspace is periodically "refreshed" to [x] with an FP64
// product H64 x.  Right after a refresh the residual and theta are FP64
// quantities, and only then is convergence accepted.  Later reduced-precision
// directions enter with weights of the order of the remaining error, so their
// product error is second order and the iteration keeps converging.  A solve
// starts with a refresh (one FP64 product), so a state that is already
// converged costs a single FP64 product.
//
// With `lock` (a normalised device vector, the first state) the search runs in
// its orthogonal complement: the guess and every correction are
// orthogonalised against it and the residual is projected, which gives the
// second eigenpair.  `psi` holds the guess on entry and the result on exit.
dmrg_status Engine::davidson(Bond& B, Buf& psi, const double* lock, double* theta_out, int64_t* nlo,
                             int64_t* n64, bool* conv) {
    const int64_t n = B.dim;
    const int kmax = std::max(2, std::min(32, opt_.davidson_max_subspace));
    TRY(ensure_dv(n, kmax));
    double* Vm = dv_V_.d();
    double* Wm = dv_W_.d();
    double* G = dv_small_.d();          // kmax x kmax at ld 32
    double* s = G + 32 * 32;            // 32
    double* sc = s + 32;                // scalars: 0 theta, 1 |r|^2, 2 |t|^2, 3 |x|^2
    double* cc = sc + 8;                // 32 (projection coefficients)
    const int ldg = 32;
    const int lowp = force_fp64_ ? dmrgdev::P_F64
                     : opt_.precision == DMRG_MIXED_FP32 ? dmrgdev::P_F32
                     : opt_.precision == DMRG_MIXED_BF16 ? dmrgdev::P_BF16 : dmrgdev::P_F64;
    const bool mixed = lowp != dmrgdev::P_F64;
    const int max_refresh = 8;
    *nlo = 0;
    *n64 = 0;
    *conv = false;
    int refreshes = 0;
    bool exact = true;        // every W column is an FP64 product
    // v -= (lock . v) lock
    auto deflate = [&](double* v) -> dmrg_status {
        if (!lock) return DMRG_OK;
        DEV(dmrgdev::dots(dev_, lock, 0, 1, v, n, sc + 4));
        DEV(dmrgdev::combine(dev_, lock, 0, 1, sc + 4, -1.0, n, v, 1));
        return DMRG_OK;
    };
    if (lock) {   // a guess inside the locked direction is replaced by the hash-random start
        TRY(deflate(psi.d()));
        DEV(dmrgdev::dots(dev_, psi.d(), 0, 1, psi.d(), n, sc + 3));
        double g2 = 0.0;
        DEV(dmrgdev::d2h(dev_, &g2, sc + 3, sizeof(double)));
        if (!(std::sqrt(std::max(g2, 0.0)) >= 1e-10)) {
            TRY(random_psi(B, psi));
            TRY(deflate(psi.d()));
        }
    }
    // V0 = psi / |psi|, W0 = H64 V0
    DEV(dmrgdev::dots(dev_, psi.d(), 0, 1, psi.d(), n, sc + 3));
    DEV(dmrgdev::copy_scaled_inv_norm(dev_, psi.d(), n, sc + 3, Vm));
    TRY(heff(B, Vm, Wm, dmrgdev::P_F64));
    *n64 += 1;
    int k = 1;
    DEV(dmrgdev::dots(dev_, Vm, n, 1, Wm, n, G));
    double theta = 0.0, rn = 0.0, prev_rn = 1e300;
    int stall = 0;
    const double tol = opt_.davidson_tol;
    // reduced-precision residuals are trusted down to about rho times the last FP64 residual
    const double rho = lowp == dmrgdev::P_BF16 ? 1e-2 : 1e-5;
    double r_exact = 1e300;
    while (true) {
        DEV(dmrgdev::small_eigh(dev_, G, k, ldg, sc, s));
        DEV(dmrgdev::combine(dev_, Vm, n, k, s, 1.0, n, dv_x_.d(), 0));
        DEV(dmrgdev::combine(dev_, Wm, n, k, s, 1.0, n, dv_hx_.d(), 0));
        DEV(dmrgdev::residual(dev_, dv_hx_.d(), dv_x_.d(), sc, n, dv_r_.d(), sc + 1));
        if (lock) {   // projected residual
            TRY(deflate(dv_r_.d()));
            DEV(dmrgdev::dots(dev_, dv_r_.d(), 0, 1, dv_r_.d(), n, sc + 1));
        }
        double hs[2];
        DEV(dmrgdev::d2h(dev_, hs, sc, 2 * sizeof(double)));
        theta = hs[0];
        rn = std::sqrt(std::max(hs[1], 0.0));
        const int64_t nprod = *nlo + *n64;
#ifdef DMRG_TRACE
        fprintf(stderr, "   dav k=%d exact=%d rn=%.3e theta=%.12f lo=%lld 64=%lld\n", k, (int)exact, rn, theta, (long long)*nlo, (long long)*n64);
#endif
        if (exact && rn <= tol) {
            *conv = true;
            break;
        }
        if (exact) r_exact = rn;
        if (nprod >= opt_.davidson_max_iter) break;
        if (mixed && !exact) {
            stall = rn > 0.8 * prev_rn ? stall + 1 : 0;
            prev_rn = rn;
            if (rn <= std::max(tol, rho * r_exact) || stall >= 3) {
                // FP64 refresh: V = [x], W = [H64 x]
                DEV(dmrgdev::dots(dev_, dv_x_.d(), 0, 1, dv_x_.d(), n, sc + 3));
                DEV(dmrgdev::copy_scaled_inv_norm(dev_, dv_x_.d(), n, sc + 3, Vm));
                TRY(heff(B, Vm, Wm, dmrgdev::P_F64));
                *n64 += 1;
                k = 1;
                DEV(dmrgdev::dots(dev_, Vm, n, 1, Wm, n, G));
                exact = true;
                stall = 0;
                prev_rn = 1e300;
                ++refreshes;
                continue;
            }
        }
        DEV(dmrgdev::precond(dev_, dv_r_.d(), B.diag.d(), sc, n, dv_t_.d()));
        if (k >= kmax) {
            DEV(dmrgdev::dots(dev_, dv_x_.d(), 0, 1, dv_x_.d(), n, sc + 3));
            DEV(dmrgdev::copy_scaled_inv_norm(dev_, dv_x_.d(), n, sc + 3, Vm));
            if (mixed && !exact) {
                // restart as a refresh: the kept column becomes an FP64 product
                TRY(heff(B, Vm, Wm, dmrgdev::P_F64));
                *n64 += 1;
                exact = true;
                ++refreshes;
                k = 1;
                DEV(dmrgdev::dots(dev_, Vm, n, 1, Wm, n, G));
                continue;
            }
            DEV(dmrgdev::copy_scaled_inv_norm(dev_, dv_hx_.d(), n, sc + 3, Wm));
            k = 1;
            DEV(dmrgdev::dots(dev_, Vm, n, 1, Wm, n, G));
        }
        DEV(dmrgdev::dots(dev_, dv_t_.d(), 0, 1, dv_t_.d(), n, sc + 2));
        DEV(dmrgdev::scale_inv_norm(dev_, dv_t_.d(), n, sc + 2));
        for (int pass = 0; pass < 2; ++pass) {
            TRY(deflate(dv_t_.d()));
            DEV(dmrgdev::dots(dev_, Vm, n, k, dv_t_.d(), n, cc));
            DEV(dmrgdev::combine(dev_, Vm, n, k, cc, -1.0, n, dv_t_.d(), 1));
        }
        DEV(dmrgdev::dots(dev_, dv_t_.d(), 0, 1, dv_t_.d(), n, sc + 2));
        double tn2;
        DEV(dmrgdev::d2h(dev_, &tn2, sc + 2, sizeof(double)));
        if (std::sqrt(std::max(tn2, 0.0)) < 1e-12) {
            if (mixed && !exact) {
                stall = 2;
                prev_rn = 0.0;
                continue;
            }
            break;
        }
        DEV(dmrgdev::copy_scaled_inv_norm(dev_, dv_t_.d(), n, sc + 2, Vm + (size_t)k * n));
        // reduced precision while refreshes last and half the product budget is
        // left; after that the solve finishes as a plain FP64 Davidson
        const bool low = mixed && refreshes < max_refresh && *nlo + *n64 < opt_.davidson_max_iter / 2;
        TRY(heff(B, Vm + (size_t)k * n, Wm + (size_t)k * n, low ? lowp : dmrgdev::P_F64));
        (low ? *nlo : *n64) += 1;
        if (low) exact = false;
        // new row of the projected matrix: G[k][a] = (H v_a)^T v_k, a <= k.  Coupling a
        // new vector through the earlier vectors' products keeps the couplings to an
        // FP64-refreshed x exact in the mixed modes; only the lower triangle is used.
        DEV(dmrgdev::dots(dev_, Wm, n, k + 1, Vm + (size_t)k * n, n, G + (size_t)k * ldg));
        ++k;
    }
    // psi <- x normalised
    DEV(dmrgdev::dots(dev_, dv_x_.d(), 0, 1, dv_x_.d(), n, sc + 3));
    DEV(dmrgdev::copy_scaled_inv_norm(dev_, dv_x_.d(), n, sc + 3, psi.d()));
    if (!exact) {
        // Stopped (product limit or stagnation) with reduced-precision
        // columns in the subspace: theta is then not an FP64 quantity.  One
        // more FP64 product gives the Rayleigh quotient of the returned vector.
        TRY(heff(B, psi.d(), Wm, dmrgdev::P_F64));
        *n64 += 1;
        DEV(dmrgdev::dots(dev_, psi.d(), 0, 1, Wm, n, sc));
        DEV(dmrgdev::d2h(dev_, &theta, sc, sizeof(double)));
    }
    *theta_out = theta;
    return DMRG_OK;
}

// ====================================================== random start
dmrg_status Engine::random_psi(Bond& B, Buf& out) {
    std::vector<double> h(B.dim);
    for (size_t x = 0; x < B.pm_S.size(); ++x) {
        const QN& q = B.S.mq[B.pm_S[x]];
        int ds = B.S.md[B.pm_S[x]], de = B.E.md[B.pm_E[x]];
        for (int a = 0; a < ds; ++a)
            for (int b = 0; b < de; ++b)
                h[B.poff[x] + (int64_t)a * de + b] =
                    2.0 * u01(hkey({(int64_t)opt_.seed, 3, q.np, q.nn, q.tm, a, b})) - 1.0;
    }
    return upload(out, h);
}

// Selection isometry per sector: keep counts by integer largest remainder
// (ties to the smaller sector), kept states = smallest SplitMix64 keys, in
// index order; optionally multiplied by a hash-random Householder reflection.
std::vector<std::vector<double>> Engine::selection_iso(const std::vector<int>& dims, int D, int tag, int pos,
                                                       const std::vector<QN>& qs, bool mix,
                                                       std::vector<int>& kept,
                                                       std::vector<std::vector<int>>* chosen_out) {
    int64_t total = 0;
    for (int d : dims) total += d;
    size_t ns = dims.size();
    kept.assign(ns, 0);
    if (total <= D) {
        for (size_t x = 0; x < ns; ++x) kept[x] = dims[x];
    } else {
        std::vector<int64_t> rem(ns);
        int64_t sum = 0;
        for (size_t x = 0; x < ns; ++x) {
            kept[x] = (int)(((int64_t)D * dims[x]) / total);
            rem[x] = ((int64_t)D * dims[x]) % total;
            sum += kept[x];
        }
        std::vector<size_t> ord(ns);
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
            if (rem[a] != rem[b]) return rem[a] > rem[b];
            return qs[a] < qs[b];
        });
        int64_t left = D - sum;
        for (size_t y = 0; y < ns && left > 0; ++y) {
            size_t x = ord[y];
            if (kept[x] < dims[x]) {
                kept[x]++;
                left--;
            }
        }
    }
    std::vector<std::vector<double>> iso(ns);
    if (chosen_out) chosen_out->assign(ns, {});
    for (size_t x = 0; x < ns; ++x) {
        int d = dims[x], k = kept[x];
        if (k == 0) continue;
        const QN& q = qs[x];
        std::vector<std::pair<uint64_t, int>> keys(d);
        for (int r = 0; r < d; ++r) keys[r] = {hkey({(int64_t)opt_.seed, tag, pos, q.np, q.nn, q.tm, r}), r};
        std::sort(keys.begin(), keys.end());
        std::vector<int> ch(k);
        for (int c = 0; c < k; ++c) ch[c] = keys[c].second;
        std::sort(ch.begin(), ch.end());
        std::vector<double> U((size_t)d * k, 0.0);
        for (int c = 0; c < k; ++c) U[(size_t)ch[c] * k + c] = 1.0;
        if (mix && d > 1) {
            std::vector<double> v(d);
            double vv = 0.0;
            for (int r = 0; r < d; ++r) {
                v[r] = 2.0 * u01(hkey({(int64_t)opt_.seed, 4, pos, q.np, q.nn, q.tm, r})) - 1.0;
                vv += v[r] * v[r];
            }
            double f = 2.0 / vv;
            for (int r = 0; r < d; ++r)
                for (int c = 0; c < k; ++c) U[(size_t)r * k + c] -= f * v[r] * v[ch[c]];
        }
        iso[x] = std::move(U);
        if (chosen_out) (*chosen_out)[x] = ch;
    }
    return iso;
}

// CI-DEAS environment block (the block-state paragraph cites a CI-based,
// dynamically extended active space grown by the orbital entropy profile).
// The block R = sites lo..N-1 keeps determinants of its composite basis (site
// lo times the block built before it, whose states are determinants): those
// differing from the reference determinant only on its k most entropic sites
// (decreasing one-orbital entropy, ties to the lower position), for the
// largest k whose CI space holds at most D determinants, completed to D from
// the next space with the fewest differing sites first, then the SplitMix64
// key (seed, 5, lo, low and high 32 bits of the determinant).  Kept rows are
// in basis order; the isometry is a selection.
std::vector<std::vector<double>> Engine::cideas_iso(const Enl& comp, const Stored& base, int D, int lo,
                                                    std::vector<int>& kept,
                                                    std::vector<std::vector<int>>& chosen) {
    const size_t ns = comp.mq.size();
    std::vector<int> rank(N_, 0);   // 1-based rank among the block's sites by entropy
    {
        std::vector<int> sites;
        for (int i = lo; i < N_; ++i) sites.push_back(i);
        std::stable_sort(sites.begin(), sites.end(),
                         [&](int a, int b) { return cd_s_[a] != cd_s_[b] ? cd_s_[a] > cd_s_[b] : a < b; });
        for (size_t k = 0; k < sites.size(); ++k) rank[sites[k]] = (int)k + 1;
    }
    const uint64_t mask = (N_ >= 64 ? ~0ull : ((1ull << N_) - 1)) & ~((1ull << lo) - 1);
    struct Cand {
        int level, pc;
        uint64_t key;
        int m, row;
    };
    std::vector<Cand> cand;
    for (size_t m = 0; m < ns; ++m) {
        int row = 0;
        for (int sg = 0; sg < 2; ++sg) {
            const int si = comp.msub[m][sg];
            if (si < 0) continue;
            for (uint64_t c0 : base.cfg[comp.sub[si].base]) {
                const uint64_t c = c0 | (sg ? (1ull << lo) : 0ull);
                const uint64_t d = (c ^ cd_ref_) & mask;
                int level = 0;
                for (int i = lo; i < N_; ++i)
                    if ((d >> i) & 1ull) level = std::max(level, rank[i]);
                const uint64_t key = hkey({(int64_t)opt_.seed, 5, lo, (int64_t)(c & 0xffffffffull), (int64_t)(c >> 32)});
                cand.push_back({level, __builtin_popcountll(d), key, (int)m, row++});
            }
        }
    }
    std::vector<char> keep(cand.size(), 0);
    if ((int64_t)cand.size() <= D) {
        std::fill(keep.begin(), keep.end(), 1);
    } else {
        std::vector<int64_t> count(N_ - lo + 2, 0);
        for (const Cand& c : cand) count[c.level]++;
        int kstar = -1;
        int64_t cum = 0;
        for (int k = 0; k <= N_ - lo; ++k) {
            if (cum + count[k] > D) break;
            cum += count[k];
            kstar = k;
        }
        std::vector<size_t> nxt;
        for (size_t x = 0; x < cand.size(); ++x) {
            if (cand[x].level <= kstar) keep[x] = 1;
            else if (cand[x].level == kstar + 1) nxt.push_back(x);
        }
        std::sort(nxt.begin(), nxt.end(), [&](size_t a, size_t b) {
            if (cand[a].pc != cand[b].pc) return cand[a].pc < cand[b].pc;
            return cand[a].key < cand[b].key;
        });
        for (size_t y = 0; y < nxt.size() && cum < D; ++y, ++cum) keep[nxt[y]] = 1;
    }
    kept.assign(ns, 0);
    chosen.assign(ns, {});
    for (size_t x = 0; x < cand.size(); ++x)
        if (keep[x]) chosen[cand[x].m].push_back(cand[x].row);
    std::vector<std::vector<double>> iso(ns);
    for (size_t m = 0; m < ns; ++m) {
        auto& ch = chosen[m];
        std::sort(ch.begin(), ch.end());
        const int d = comp.md[m], k = (int)ch.size();
        kept[m] = k;
        if (!k) continue;
        std::vector<double> U((size_t)d * k, 0.0);
        for (int c = 0; c < k; ++c) U[(size_t)ch[c] * k + c] = 1.0;
        iso[m] = std::move(U);
    }
    return iso;
}

dmrg_status Engine::set_cideas(const double* s1, const double* n1) {
    if (!loaded_) return fail(DMRG_ERR_STATE, "no Hamiltonian loaded");
    if (!s1 && !n1) {
        cideas_ = false;
        init_ = false;
        return DMRG_OK;
    }
    if (!s1 || !n1) return fail(DMRG_ERR_ARG, "give both the entropies and the occupations, or neither");
    // measured values carry rounding (an occupation of 1 + 4e-16); only their order is used
    const double slack = 1e-9;
    for (int i = 0; i < N_; ++i)
        if (!std::isfinite(s1[i]) || s1[i] < -slack || !std::isfinite(n1[i]) || n1[i] < -slack ||
            n1[i] > 1.0 + slack)
            return fail(DMRG_ERR_ARG, "entropies must be finite and >= 0, occupations in [0, 1] (within 1e-9)");
    cds_site_.assign(s1, s1 + N_);
    cdn_site_.assign(n1, n1 + N_);
    cideas_ = true;
    init_ = false;   // the next sweep starts from CI-DEAS blocks
    return DMRG_OK;
}

// chain-position profile and reference determinant of the CI-DEAS start
void Engine::cideas_chain() {
    cd_s_.assign(N_, 0.0);
    std::vector<double> occ(N_);
    for (int a = 0; a < N_; ++a) {
        cd_s_[a] = cds_site_[order_[a]];
        occ[a] = cdn_site_[order_[a]];
    }
    cd_ref_ = 0;
    for (int sp = 0; sp < 2; ++sp) {
        std::vector<int> sites;
        for (int a = 0; a < N_; ++a)
            if ((sp == 0) == (delta_[a].np == 1)) sites.push_back(a);
        std::stable_sort(sites.begin(), sites.end(),
                         [&](int a, int b) { return occ[a] != occ[b] ? occ[a] > occ[b] : a < b; });
        const int cnt = sp == 0 ? T_.np : T_.nn;
        for (int x = 0; x < cnt && x < (int)sites.size(); ++x) cd_ref_ |= 1ull << sites[x];
    }
}

// ============================================================ initialise
dmrg_status Engine::initialize(int D) {
    if (cideas_) cideas_chain();
    cur_.reset();
    psi_.reset();
    psi1_.reset();
    L_.clear();
    R_.clear();
    L_.resize(N_ + 1);
    R_.resize(N_ + 2);
    L_[0] = vacuum('L', 0);
    R_[N_] = vacuum('R', N_);
    if (!L_[0] || !R_[N_]) return fail(DMRG_ERR_OUT_OF_MEMORY, "vacuum block");
    for (int lo = N_ - 1; lo >= 2; --lo) {
        const Stored& base = *R_[lo + 1];
        std::set<QN> cand;
        for (int sg = 0; sg < 2; ++sg)
            for (const QN& q : base.basis.q) cand.insert(sg ? q + delta_[lo] : q);
        std::vector<QN> allowed;
        for (const QN& q : cand)
            if (reachable(pre_[lo], T_ - q)) allowed.push_back(q);
        auto blk = std::make_unique<Stored>();
        blk->side = 'R';
        blk->lo = lo;
        blk->hi = N_;
        OpSet eops;
        TRY(enlarge(base, 'R', allowed, blk->comp, eops));
        std::vector<int> kept;
        std::vector<std::vector<int>> chosen;
        auto iso = cideas_ ? cideas_iso(blk->comp, base, D, lo, kept, chosen)
                           : selection_iso(blk->comp.md, D, 1, lo, blk->comp.mq, !opt_.select_basis, kept, &chosen);
        std::vector<int> keep_m, kdim;
        std::vector<double> flat;
        for (size_t m = 0; m < kept.size(); ++m) {
            if (!kept[m]) continue;
            keep_m.push_back((int)m);
            kdim.push_back(kept[m]);
            blk->basis.add(blk->comp.mq[m], kept[m]);
            blk->comp_m.push_back((int)m);
            blk->iso_off.push_back((int64_t)flat.size());
            flat.insert(flat.end(), iso[m].begin(), iso[m].end());
            size_t pad = (32 - flat.size() % 32) % 32;
            flat.insert(flat.end(), pad, 0.0);
        }
        TRY(upload(blk->iso, flat));
        bool normal_in = !normal_S(lo - 1);
        TRY(renormalize(blk->comp, eops, normal_in, *blk, keep_m, kdim));
        if ((opt_.select_basis || cideas_) && base.has_cfg) {
            blk->has_cfg = true;
            for (size_t x = 0; x < keep_m.size(); ++x) {
                int m = keep_m[x];
                std::vector<uint64_t> comp;
                for (int sg = 0; sg < 2; ++sg) {
                    int si = blk->comp.msub[m][sg];
                    if (si < 0) continue;
                    for (uint64_t c : base.cfg[blk->comp.sub[si].base])
                        comp.push_back(c | (sg ? (1ull << lo) : 0ull));
                }
                std::vector<uint64_t> v;
                for (int r : chosen[m]) v.push_back(comp[r]);
                blk->cfg.push_back(v);
            }
        }
        R_[lo] = std::move(blk);
    }
    init_ = true;
    dir_ = 0;
    bond_ = 0;
    fresh_ = false;
    sweeps_done_ = 0;
    have_prev_sweep_ = false;
    TRY(setup_bond(0, cur_));
    TRY(random_psi(*cur_, psi_));
    if (opt_.n_states == 2) TRY(random_psi(*cur_, psi1_));
    return DMRG_OK;
}

// ===================================================== density matrix
// rho of the S (left = true) or E sectors present in psi, with the
// perturbation alpha * sum_O (O psi)(O psi)^T over c+ and c of the block's
// sites.  rho blocks are dense (d x d) at roff[x] for psi block x.
dmrg_status Engine::density_matrix(Bond& B, const Buf& psi, double weight, int beta, bool left, double alpha,
                                   Buf& rho, const std::vector<int64_t>& roff, const std::vector<int>& rld) {
    const Enl &S = B.S, &E = B.E;
    int nb = (int)B.pm_S.size();
    std::vector<int> rdim(nb);
    for (int x = 0; x < nb; ++x) rdim[x] = left ? S.md[B.pm_S[x]] : E.md[B.pm_E[x]];
    // bufs: 0 psi, 1 ops, 2 Phi, 3 rho
    std::vector<std::vector<GemmChunk>> lists(nb);
    GB g1;
    int64_t phi = 0;
    for (int x = 0; x < nb; ++x) {
        int ds = S.md[B.pm_S[x]], de = E.md[B.pm_E[x]];
        if (left) lists[x].push_back(GemmChunk{weight, B.poff[x], B.poff[x], de, de, de, 0, 0, 0, 1});
        else lists[x].push_back(GemmChunk{weight, B.poff[x], B.poff[x], de, de, ds, 0, 0, 1, 0});
    }
    if (alpha != 0.0) {
        const OpSet& ops = left ? B.Sops : B.Eops;
        const Enl& en = left ? S : E;
        int lo = left ? 0 : B.b + 1, hi = left ? B.b + 1 : N_;
        for (int site = lo; site < hi; ++site) {
            const Op* C = ops.get({'C', site, 0});
            if (!C) continue;
            for (int tr = 0; tr < 2; ++tr) {
                // Phi = op(C) psi (left: rows; right: columns), per psi block
                for (int x = 0; x < nb; ++x) {
                    int mS = B.pm_S[x], mE = B.pm_E[x];
                    int m_in = left ? mS : mE;
                    int ds = S.md[mS], de = E.md[mE];
                    // output merged sector of op(C) on m_in
                    int m_out = -1;
                    for (int i : en.msub[m_in]) {
                        if (i < 0) continue;
                        for (int q : C->acting(i, tr)) m_out = en.sub[tr ? C->blk[q].in : C->blk[q].out].m;
                    }
                    if (m_out < 0) continue;
                    int x2 = left ? B.blk_of_S[m_out] : -1;
                    if (!left) {
                        int ms2 = S.find_m(T_ - E.mq[m_out]);
                        x2 = ms2 >= 0 ? B.blk_of_S[ms2] : -1;
                    }
                    if (x2 < 0) continue;
                    int dout = en.md[m_out];
                    int rows = left ? dout : ds, cols = left ? de : dout;
                    int64_t po = phi;
                    phi += ((int64_t)rows * cols + 31) / 32 * 32;
                    // every sub-row (left) / sub-column (right) of Phi: chunks over input subs
                    for (int o : en.msub[m_out]) {
                        if (o < 0) continue;
                        g1.begin();
                        for (int i : en.msub[m_in]) {
                            if (i < 0) continue;
                            for (int q : C->acting(i, tr)) {
                            const Blk* b = &C->blk[q];
                            if ((tr ? b->in : b->out) != o) continue;
                            if (left)
                                g1.chunk(1.0, 1, b->off, b->cols, tr, 0, B.poff[x] + (int64_t)en.sub[i].off * de, de,
                                         false, en.sub[i].dim);
                            else
                                g1.chunk(1.0, 0, B.poff[x] + en.sub[i].off, de, false, 1, b->off, b->cols, !tr,
                                         en.sub[i].dim);
                            }
                        }
                        if (left) g1.end(2, po + (int64_t)en.sub[o].off * cols, cols, en.sub[o].dim, cols, 0);
                        else g1.end(2, po + en.sub[o].off, cols, rows, en.sub[o].dim, 0);
                    }
                    if (left) lists[x2].push_back(GemmChunk{alpha * weight, po, po, cols, cols, cols, 2, 2, 0, 1});
                    else lists[x2].push_back(GemmChunk{alpha * weight, po, po, cols, cols, rows, 2, 2, 1, 0});
                }
            }
        }
    }
    GB g2;
    for (int x = 0; x < nb; ++x) {
        g2.begin();
        for (auto& c : lists[x]) g2.chunks.push_back(c);
        g2.end(3, roff[x], rld[x], rdim[x], rdim[x], beta);
    }
    Buf phib;
    TRY(alloc_buf(phib, std::max<int64_t>(phi, 1) * sizeof(double)));
    GemmPlan p1, p2;
    TRY(finish_plan(*this, g1, p1));
    TRY(finish_plan(*this, g2, p2));
    const OpSet& ops = left ? B.Sops : B.Eops;
    BufTable bufs{psi.p, ops.pool.p, phib.p, rho.p};
    TRY(run_gemm(dmrgdev::P_F64, bufs, p1));
    TRY(run_gemm(dmrgdev::P_F64, bufs, p2));
    return DMRG_OK;
}

// ================================================ truncate + next bond
dmrg_status Engine::truncate_and_move(int D, double alpha, double* disc) {
    Bond& B = *cur_;
    const bool left = dir_ == 0;
    const int b = B.b;
    const Enl& en = left ? B.S : B.E;
    int nb = (int)B.pm_S.size();
    // merged sectors of en present in psi, in en order
    std::vector<int> pm(nb);
    for (int x = 0; x < nb; ++x) pm[x] = left ? B.pm_S[x] : B.pm_E[x];
    std::vector<int> mpos(en.mq.size(), -1);   // merged -> psi block
    for (int x = 0; x < nb; ++x) mpos[pm[x]] = x;
    std::vector<int> keep_m, kdim;
    std::vector<double> flat;
    std::vector<int64_t> iso_off;
    std::vector<std::vector<int>> chosen;
    *disc = 0.0;
    auto blk = std::make_unique<Stored>();
    blk->side = left ? 'L' : 'R';
    blk->lo = left ? 0 : b + 1;
    blk->hi = left ? b + 1 : N_;
    if (opt_.select_basis) {
        std::vector<int> dims;
        std::vector<QN> qs;
        std::vector<int> ms;
        for (size_t m = 0; m < en.mq.size(); ++m)
            if (mpos[m] >= 0) {
                dims.push_back(en.md[m]);
                qs.push_back(en.mq[m]);
                ms.push_back((int)m);
            }
        std::vector<int> kept;
        auto iso = selection_iso(dims, D, left ? 2 : 1, b + 1, qs, false, kept, &chosen);
        std::vector<std::vector<int>> ch2;
        for (size_t y = 0; y < ms.size(); ++y) {
            if (!kept[y]) continue;
            keep_m.push_back(ms[y]);
            kdim.push_back(kept[y]);
            iso_off.push_back((int64_t)flat.size());
            flat.insert(flat.end(), iso[y].begin(), iso[y].end());
            flat.insert(flat.end(), (32 - flat.size() % 32) % 32, 0.0);
            ch2.push_back(chosen[y]);
        }
        chosen = ch2;
        TRY(upload(blk->iso, flat));
    } else {
        // sector density matrices in padded slots grouped by size; one batched
        // eigensolver call per size
        std::vector<int> rdim(nb), rld(nb), slot(nb);
        std::vector<int64_t> roff(nb), woff(nb);
        std::map<int, std::vector<int>> buckets;
        for (int x = 0; x < nb; ++x) {
            rdim[x] = left ? B.S.md[B.pm_S[x]] : B.E.md[B.pm_E[x]];
            static const int sizes[] = {8, 16, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048,
                                        3072, 4096, 6144, 8192};
            int P = rdim[x];
            for (int z : sizes)
                if (z >= rdim[x]) {
                    P = z;
                    break;
                }
            rld[x] = P;
            buckets[P].push_back(x);
        }
        int64_t tot = 0, wtot = 0;
        std::vector<std::array<int64_t, 4>> bk;   // P, count, A offset, w offset
        std::vector<int32_t> nlist;
        std::vector<int64_t> nlist_off;
        for (auto& kv : buckets) {
            const int P = kv.first;
            bk.push_back({P, (int64_t)kv.second.size(), tot, wtot});
            nlist_off.push_back((int64_t)nlist.size());
            for (size_t q = 0; q < kv.second.size(); ++q) {
                int x = kv.second[q];
                slot[x] = (int)q;
                roff[x] = tot + (int64_t)q * P * P;
                woff[x] = wtot + (int64_t)q * P + (P - rdim[x]);   // real eigenvalues are the last n
                nlist.push_back(rdim[x]);
            }
            tot += (int64_t)P * P * kv.second.size();
            wtot += (int64_t)P * kv.second.size();
        }
        Buf rho, w, nbuf;
        TRY(alloc_buf(rho, std::max<int64_t>(tot, 1) * sizeof(double)));
        TRY(alloc_buf(w, std::max<int64_t>(wtot, 1) * sizeof(double)));
        TRY(upload(nbuf, nlist));
        for (size_t y = 0; y < bk.size(); ++y)
            DEV(dmrgdev::pad_init(dev_, rho.d() + bk[y][2], (int)bk[y][0], (int)bk[y][1],
                                  nbuf.as<int32_t>() + nlist_off[y]));
        double td = now();
        if (opt_.n_states == 2) {   // the two states' density matrices, averaged
            TRY(density_matrix(B, psi_, 0.5, 0, left, alpha, rho, roff, rld));
            TRY(density_matrix(B, psi1_, 0.5, 1, left, alpha, rho, roff, rld));
        } else {
            TRY(density_matrix(B, psi_, 1.0, 0, left, alpha, rho, roff, rld));
        }
        acc_.density_seconds += now() - td;
        td = now();
        {
            std::vector<int> bP, bc;
            std::vector<int64_t> ba, bw;
            for (auto& b4 : bk) {
                bP.push_back((int)b4[0]);
                bc.push_back((int)b4[1]);
                ba.push_back(b4[2]);
                bw.push_back(b4[3]);
            }
            DEV(dmrgdev::syevd_buckets(dev_, (int)bk.size(), bP.data(), bc.data(), rho.d(), ba.data(), w.d(),
                                       bw.data()));
        }
        std::vector<double> hwall(wtot);
        DEV(dmrgdev::d2h(dev_, hwall.data(), w.p, wtot * sizeof(double)));
        // compact the real eigenvalues: block x owns hw[woff[x] .. woff[x] + rdim[x])
        std::vector<double> hw;
        for (int x = 0; x < nb; ++x) {
            const int64_t src = woff[x];
            woff[x] = (int64_t)hw.size();
            hw.insert(hw.end(), hwall.begin() + src, hwall.begin() + src + rdim[x]);
        }
        double tr = 0.0;
        for (double v : hw) tr += v;
        struct Wt {
            double w;
            int x, e;
        };
        std::vector<Wt> all;
        // listed by sector, eigenvalues ascending within a sector; the stable sort keeps
        // equal weights in that order
        for (int x = 0; x < nb; ++x)
            for (int e = 0; e < rdim[x]; ++e) all.push_back({hw[woff[x] + e] / tr, x, e});
        std::stable_sort(all.begin(), all.end(), [](const Wt& a, const Wt& c) { return a.w > c.w; });
        int64_t cnt = (int64_t)all.size();
        int64_t nk = std::min<int64_t>(D, cnt);
        if (opt_.trunc_eps > 0.0) {
            // DBSS: the fewest weights whose discarded remainder is at most
            // trunc_eps (summed in descending order), within [d_min, D]
            int64_t n = 0;
            double kw = 0.0;
            while (n < cnt && 1.0 - kw > opt_.trunc_eps) kw += all[n++].w;
            nk = std::min<int64_t>(std::min<int64_t>(std::max<int64_t>(n, opt_.d_min), D), cnt);
        }
        const int64_t n0 = nk;
        while (nk > 0 && nk < cnt && all[nk - 1].w - all[nk].w <= opt_.tie_tol) --nk;
        if (nk == 0) {
            nk = n0;
            while (nk < cnt && all[nk - 1].w - all[nk].w <= opt_.tie_tol) ++nk;
        }
        double kept_w = 0.0;
        std::vector<std::vector<int>> sel(nb);
        for (int64_t y = 0; y < nk; ++y) {
            kept_w += all[y].w;
            sel[all[y].x].push_back(all[y].e);
        }
        *disc = std::max(0.0, 1.0 - kept_w);
        // U per kept sector: eigenvectors in descending weight order
        Buf idxb;
        std::vector<int32_t> idx;
        std::vector<std::array<int64_t, 3>> jobs;   // x, idx offset, k
        int64_t utot = 0;
        for (size_t m = 0; m < en.mq.size(); ++m) {
            int x = mpos[m];
            if (x < 0 || sel[x].empty()) continue;
            auto& s = sel[x];
            std::sort(s.begin(), s.end(), [&](int a, int c) { return hw[woff[x] + a] > hw[woff[x] + c]; });
            keep_m.push_back((int)m);
            kdim.push_back((int)s.size());
            iso_off.push_back(utot);
            jobs.push_back({x, (int64_t)idx.size(), (int64_t)s.size()});
            for (int e : s) idx.push_back(e + (rld[x] - rdim[x]));   // eigenvector row in the padded slot
            utot += ((int64_t)rdim[x] * s.size() + 31) / 32 * 32;
        }
        TRY(upload(idxb, idx));
        TRY(alloc_buf(blk->iso, std::max<int64_t>(utot, 1) * sizeof(double)));
        for (size_t y = 0; y < jobs.size(); ++y) {
            int x = (int)jobs[y][0];
            DEV(dmrgdev::gather_evecs(dev_, rho.d() + roff[x], rdim[x], rld[x], idxb.as<int32_t>() + jobs[y][1],
                                      (int)jobs[y][2], blk->iso.d() + iso_off[y]));
        }
        acc_.eig_seconds += now() - td;
    }
    int64_t kept_tot = 0;
    for (size_t y = 0; y < keep_m.size(); ++y) {
        blk->basis.add(en.mq[keep_m[y]], kdim[y]);
        blk->comp_m.push_back(keep_m[y]);
        kept_tot += kdim[y];
    }
    acc_.kept_max = std::max<int64_t>(acc_.kept_max, kept_tot);
    blk->iso_off = iso_off;
    blk->comp = en;
    bool normal_in = left ? normal_S(b) : !normal_S(b);
    double trn = now();
    TRY(renormalize(en, left ? B.Sops : B.Eops, normal_in, *blk, keep_m, kdim));
    acc_.renormalize_seconds += now() - trn;
    const Stored& base = left ? *L_[b] : *R_[b + 2];
    if (opt_.select_basis && base.has_cfg) {
        blk->has_cfg = true;
        for (size_t y = 0; y < keep_m.size(); ++y) {
            int m = keep_m[y];
            std::vector<uint64_t> comp;
            for (int sg = 0; sg < 2; ++sg) {
                int si = en.msub[m][sg];
                if (si < 0) continue;
                for (uint64_t c : base.cfg[en.sub[si].base]) comp.push_back(c | (sg ? (1ull << en.site) : 0ull));
            }
            std::vector<uint64_t> v;
            for (int r : chosen[y]) v.push_back(comp[r]);
            blk->cfg.push_back(v);
        }
    }
    // next bond and prediction
    int nbond = left ? b + 1 : b - 1;
    std::unique_ptr<Bond> NB;
    if (left) L_[b + 1] = std::move(blk);
    else R_[b + 1] = std::move(blk);
    TRY(setup_bond(nbond, NB));
    double tpr = now();
    Bond& B2 = *NB;
    const Stored& nw = left ? *L_[b + 1] : *R_[b + 1];
    // Phi: left: U_m^T psi_m (k x dE) ; right: psi_m V (dS x k)
    GB g1, g2;
    std::vector<int64_t> phoff(nb, -1);
    int64_t ph = 0;
    std::vector<int> newx(en.mq.size(), -1);
    for (size_t y = 0; y < keep_m.size(); ++y) newx[keep_m[y]] = (int)y;
    for (int x = 0; x < nb; ++x) {
        int m = pm[x];
        int y = newx[m];
        if (y < 0) continue;
        int ds = B.S.md[B.pm_S[x]], de = B.E.md[B.pm_E[x]], k = kdim[y];
        phoff[x] = ph;
        if (left) {
            ph += ((int64_t)k * de + 31) / 32 * 32;
            g1.begin();
            g1.chunk(1.0, 1, nw.iso_off[y], k, true, 0, B.poff[x], de, false, ds);
            g1.end(2, phoff[x], de, k, de, 0);
        } else {
            ph += ((int64_t)ds * k + 31) / 32 * 32;
            g1.begin();
            g1.chunk(1.0, 0, B.poff[x], de, false, 1, nw.iso_off[y], k, false, de);
            g1.end(2, phoff[x], k, ds, k, 0);
        }
    }
    // bufs: 0 psi(old), 1 new iso, 2 Phi, 3 psi(new), 4 far iso (R_{b+2} for L->R, L_b for R->L)
    const Stored& far = left ? *R_[b + 2] : *L_[b];
    int nb2 = (int)B2.pm_S.size();
    std::vector<std::vector<GemmChunk>> lists(nb2 * 4);
    auto sid = [&](int x2, int i, int j) { return x2 * 4 + B2.S.sub[i].sigma * 2 + B2.E.sub[j].sigma; };
    for (int x = 0; x < nb; ++x) {
        if (phoff[x] < 0) continue;
        int y = newx[pm[x]];
        int k = kdim[y];
        if (left) {
            // columns of Phi: E sub-sectors j = (sigma_{b+1}, R_{b+2} sector r)
            int de = B.E.md[B.pm_E[x]];
            for (int j : B.E.msub[B.pm_E[x]]) {
                if (j < 0) continue;
                const Sub& sj = B.E.sub[j];
                int i2 = B2.S.find_sub(y, sj.sigma);
                if (i2 < 0) continue;
                int x2 = B2.blk_of_S[B2.S.sub[i2].m];
                if (x2 < 0) continue;
                int r = sj.base;   // sector of R_{b+2}
                int kr = far.basis.d[r];
                int cm = far.comp_m[r];
                for (int c : far.comp.msub[cm]) {
                    if (c < 0) continue;
                    const Sub& sc = far.comp.sub[c];
                    int j2 = B2.E.find_sub(sc.base, sc.sigma);
                    if (j2 < 0 || B2.E.sub[j2].m != B2.pm_E[x2]) continue;
                    lists[sid(x2, i2, j2)].push_back(GemmChunk{1.0, phoff[x] + sj.off, far.iso_off[r] + (int64_t)sc.off * kr,
                                                               de, kr, kr, 2, 4, 0, 1});
                }
            }
        } else {
            // rows of Phi: S sub-sectors i = (L_b sector l, sigma_b)
            for (int i : B.S.msub[B.pm_S[x]]) {
                if (i < 0) continue;
                const Sub& si = B.S.sub[i];
                int j2 = B2.E.find_sub(y, si.sigma);
                if (j2 < 0) continue;
                int ms2 = B2.S.find_m(T_ - B2.E.sub[j2].q);
                if (ms2 < 0) continue;
                int x2 = B2.blk_of_S[ms2];
                if (x2 < 0) continue;
                int l = si.base;
                int kl = far.basis.d[l];
                int cm = far.comp_m[l];
                for (int c : far.comp.msub[cm]) {
                    if (c < 0) continue;
                    const Sub& sc = far.comp.sub[c];
                    int i2 = B2.S.find_sub(sc.base, sc.sigma);
                    if (i2 < 0 || B2.S.sub[i2].m != B2.pm_S[x2]) continue;
                    lists[sid(x2, i2, j2)].push_back(GemmChunk{1.0, far.iso_off[l] + (int64_t)sc.off * kl,
                                                               phoff[x] + (int64_t)si.off * k, kl, k, kl, 4, 2, 0, 0});
                }
            }
        }
    }
    for (int x2 = 0; x2 < nb2; ++x2)
        for (int i : B2.S.msub[B2.pm_S[x2]])
            for (int j : B2.E.msub[B2.pm_E[x2]]) {
                if (i < 0 || j < 0) continue;
                g2.begin();
                for (auto& c : lists[sid(x2, i, j)]) g2.chunks.push_back(c);
                int ldy = B2.E.md[B2.pm_E[x2]];
                g2.end(3, B2.poff[x2] + (int64_t)B2.S.sub[i].off * ldy + B2.E.sub[j].off, ldy, B2.S.sub[i].dim,
                       B2.E.sub[j].dim, 0);
            }
    Buf phib, npsi;
    TRY(alloc_buf(phib, std::max<int64_t>(ph, 1) * sizeof(double)));
    TRY(alloc_buf(npsi, std::max<int64_t>(B2.dim, 1) * sizeof(double)));
    GemmPlan p1, p2;
    TRY(finish_plan(*this, g1, p1));
    TRY(finish_plan(*this, g2, p2));
    BufTable bufs{psi_.p, nw.iso.p, phib.p, npsi.p, far.iso.p};
    TRY(run_gemm(dmrgdev::P_F64, bufs, p1));
    TRY(run_gemm(dmrgdev::P_F64, bufs, p2));
    Buf npsi1;   // the second state through the same plans
    if (opt_.n_states == 2) {
        TRY(alloc_buf(npsi1, std::max<int64_t>(B2.dim, 1) * sizeof(double)));
        BufTable bufs1{psi1_.p, nw.iso.p, phib.p, npsi1.p, far.iso.p};
        TRY(run_gemm(dmrgdev::P_F64, bufs1, p1));
        TRY(run_gemm(dmrgdev::P_F64, bufs1, p2));
    }
    // fall back to the hash-random start if the guess vanished
    if (!scal_.p) TRY(alloc_buf(scal_, 64 * sizeof(double)));
    DEV(dmrgdev::dots(dev_, npsi.d(), 0, 1, npsi.d(), B2.dim, scal_.d()));
    double nn = 0.0;
    DEV(dmrgdev::d2h(dev_, &nn, scal_.p, sizeof(double)));
    psi_ = std::move(npsi);
    if (!(std::sqrt(std::max(nn, 0.0)) >= 1e-10)) TRY(random_psi(B2, psi_));
    if (opt_.n_states == 2) psi1_ = std::move(npsi1);   // checked when its solve deflates it
    cur_ = std::move(NB);
    acc_.predict_seconds += now() - tpr;
    return DMRG_OK;
}

// =============================================================== sweeps
dmrg_status Engine::steps(const int32_t* ordering, int D, int64_t max_steps, bool until_sweep_end,
                          dmrg_sweep_stats* st) {
    if (!loaded_) return fail(DMRG_ERR_STATE, "no Hamiltonian loaded");
    if (D < 1) return fail(DMRG_ERR_ARG, "D must be >= 1");
    if (N_ < 2) return fail(DMRG_ERR_ARG, "need at least 2 sites for a two-site sweep");
    std::vector<int> before = order_;
    TRY(set_order(ordering));
    double t0 = now();
    if (!init_) {
        TRY(initialize(D));
        sweep_min_ = INFINITY;
        sweep_min1_ = INFINITY;
        sweep_steps_ = 0;
        acc_ = dmrg_sweep_stats{};
    }
    if (sweep_steps_ == 0) {
        acc_ = dmrg_sweep_stats{};
        sweep_min_ = INFINITY;
        sweep_min1_ = INFINITY;
        reset_measure();
    }
    TRY(ensure_dv(cur_->dim, std::max(2, std::min(32, opt_.davidson_max_subspace))));
    dmrg_status ret = DMRG_OK;
    int64_t done = 0;
    while (done < max_steps) {
        // solve at the current bond unless psi is its converged eigenvector
        if (!fresh_) {
            double th;
            int64_t nlo, n64;
            bool conv;
            const bool check = check_fp64_ && opt_.precision != DMRG_FP64;
            if (check) {   // the guess, for the FP64 repeat
                TRY(alloc_buf(chk_psi_, std::max<int64_t>(cur_->dim, 1) * sizeof(double)));
                DEV(dmrgdev::d2d(dev_, chk_psi_.p, psi_.p, cur_->dim * sizeof(double)));
            }
            heff_time_ = 0.0;
            TRY(davidson(*cur_, psi_, nullptr, &th, &nlo, &n64, &conv));
            acc_.heff_seconds += heff_time_;
            acc_.heff_flops += cur_->flops_alg * (double)(nlo + n64);
            acc_.heff_flops_executed += cur_->flops * (double)(nlo + n64);
            if (check) {
                double th64;
                int64_t a, c;
                bool cv;
                force_fp64_ = true;
                dmrg_status cs = davidson(*cur_, chk_psi_, nullptr, &th64, &a, &c, &cv);
                force_fp64_ = false;
                TRY(cs);
                acc_.check_solves += 1;
                acc_.check_max_rel = std::max(acc_.check_max_rel, std::fabs(th - th64) / std::fabs(th64));
            }
            acc_.products_low += nlo;
            acc_.products_fp64 += n64;
            acc_.solves += 1;
            if (!conv) {
                acc_.not_converged += 1;
                ret = DMRG_WARN_NOT_CONVERGED;
            }
            theta_ = th;
            if (opt_.n_states == 2) {   // the second state, in the complement of the first
                heff_time_ = 0.0;
                TRY(davidson(*cur_, psi1_, psi_.d(), &th, &nlo, &n64, &conv));
                acc_.heff_seconds += heff_time_;
                acc_.heff_flops += cur_->flops_alg * (double)(nlo + n64);
                acc_.heff_flops_executed += cur_->flops * (double)(nlo + n64);
                acc_.products_low += nlo;
                acc_.products_fp64 += n64;
                acc_.solves += 1;
                if (!conv) {
                    acc_.not_converged += 1;
                    ret = DMRG_WARN_NOT_CONVERGED;
                }
                theta1_ = th;
            }
            fresh_ = true;
        }
        sweep_min_ = std::min(sweep_min_, theta_);
        sweep_min1_ = std::min(sweep_min1_, theta1_);
        ++done;
        ++sweep_steps_;
        acc_.steps += 1;
        if (opt_.measure && dir_ == 1) {
            const double tm = now();
            TRY(measure_bond(*cur_));
            acc_.measure_seconds += now() - tm;
        }
        bool last = dir_ == 0 ? bond_ == N_ - 2 : bond_ == 0;
        if (last) {
            if (dir_ == 0) {
                dir_ = 1;   // turn: same bond, same state
            } else {
                dir_ = 0;
                sweeps_done_ += 1;
                have_energy_ = true;
                if (opt_.measure) meas_valid_ = true;
                energy_ = sweep_min_;
                acc_.energy = sweep_min_;
                acc_.energy_excited = opt_.n_states == 2 ? sweep_min1_ : 0.0;
                acc_.last_theta = theta_;
                acc_.delta_energy = have_prev_sweep_ ? sweep_min_ - prev_sweep_energy_
                                                     : std::numeric_limits<double>::quiet_NaN();
                prev_sweep_energy_ = sweep_min_;
                have_prev_sweep_ = true;
                acc_.sweep_seconds = now() - t0;
                if (st) *st = acc_;
                sweep_steps_ = 0;
                if (until_sweep_end) return ret;
                acc_ = dmrg_sweep_stats{};
                sweep_min_ = INFINITY;
                sweep_min1_ = INFINITY;
                reset_measure();
                t0 = now();
            }
            continue;
        }
        double alpha = sweeps_done_ < opt_.noise_sweeps ? opt_.noise : 0.0;
        double disc = 0.0;
        double tr0 = now();
        TRY(truncate_and_move(D, alpha, &disc));
        acc_.renorm_seconds += now() - tr0;
        acc_.discarded_max = std::max(acc_.discarded_max, disc);
        acc_.discarded_sum += disc;
        bond_ = cur_->b;
        fresh_ = false;
        TRY(ensure_dv(cur_->dim, std::max(2, std::min(32, opt_.davidson_max_subspace))));
    }
    acc_.energy = sweep_min_;
    acc_.energy_excited = opt_.n_states == 2 ? sweep_min1_ : 0.0;
    acc_.last_theta = theta_;
    acc_.delta_energy = std::numeric_limits<double>::quiet_NaN();   // the sweep is not finished
    acc_.sweep_seconds += now() - t0;
    if (st) *st = acc_;
    return ret;
}

// ================================================== orbital correlations
void Engine::reset_measure() {
    if (!opt_.measure) return;
    const size_t n2 = (size_t)N_ * N_;
    m_n1_.assign(N_, 0.0);
    m_pni_.assign(n2, 0.0);
    m_pnj_.assign(n2, 0.0);
    m_nn_.assign(n2, 0.0);
    m_hop_.assign(n2, 0.0);
    meas_valid_ = false;
}

// At bond b of the right-to-left half, with E site j = b + 1: <n_j>, and for
// every S site i <= b <n_i>, <n_i n_j> and <c+_i c_j> in the state psi (the
// inputs of rho_i and rho_ij, the entropy paragraph).  Phase 1 (grouped GEMM,
// FP64): Z = N_i psi_x per psi block, and, for i of j's species and 2m,
// T = C_i psi_x on the E columns where j is occupied.  Phase 2 (segment dot
// products): <n_i> = <psi, Z>, <n_i n_j> = <psi, Z> over the columns with j
// occupied, <n_j> likewise with psi itself, and <c+_i c_j> = sum_x
// (-1)^N(S sector of x) <psi_x2 on the columns (r, 0), T on (r, 1)>: with S
// before E in the Jordan-Wigner order and j first in E,
// c_j |s, (r, 1)> = (-1)^N(s) |s, (r, 0)>.  The i are taken in batches whose
// intermediates fit in a few copies of psi.
dmrg_status Engine::measure_bond(Bond& B) {
    const Enl &S = B.S, &E = B.E;
    const int b = B.b, j = b + 1;
    const int nb = (int)B.pm_S.size();
    const int64_t psi_elems = B.dim;
    auto esub = [&](int x, int sigma) -> const Sub* {
        if (x < 0) return nullptr;
        const int i = E.msub[B.pm_E[x]][sigma];
        return i < 0 ? nullptr : &E.sub[i];
    };
    // outputs: 0 = <n_j>; 1 + 3 i + {0, 1, 2} = <n_i>, <n_i n_j>, <c+_i c_j>
    const int nout = 1 + 3 * (b + 1);
    std::vector<std::vector<dmrgdev::SegDot>> segs_of(nout);
    auto seg = [&](int out, double coef, int abuf, int64_t aoff, int lda, int bbuf, int64_t boff, int ldb,
                   int rows, int cols) {
        if (rows <= 0 || cols <= 0) return;
        const int step = std::max(1, 32768 / cols);
        for (int r0 = 0; r0 < rows; r0 += step) {
            dmrgdev::SegDot sd{};
            sd.coef = coef;
            sd.a_off = aoff + (int64_t)r0 * lda;
            sd.b_off = boff + (int64_t)r0 * ldb;
            sd.rows = std::min(step, rows - r0);
            sd.cols = cols;
            sd.lda = lda;
            sd.ldb = ldb;
            sd.a_buf = (uint8_t)abuf;
            sd.b_buf = (uint8_t)bbuf;
            segs_of[out].push_back(sd);
        }
    };
    for (int x = 0; x < nb; ++x) {
        const Sub* e1 = esub(x, 1);
        if (!e1) continue;
        const int ds = S.md[B.pm_S[x]], de = E.md[B.pm_E[x]];
        seg(0, 1.0, 0, B.poff[x] + e1->off, de, 0, B.poff[x] + e1->off, de, ds, e1->dim);
    }
    const OpSet& ops = B.Sops;
    const int64_t cap = std::max<int64_t>(8 * psi_elems, (int64_t)1 << 24);
    Buf outb;
    TRY(alloc_buf(outb, (size_t)nout * sizeof(double)));
    for (int i0 = 0; i0 <= b;) {
        GB g;
        int64_t phi = 0;
        int i1 = i0;
        // each i needs at most two psi-sized intermediates (Z, and T)
        while (i1 <= b && (i1 == i0 || phi + 2 * psi_elems + 64 * nb <= cap)) {
            const int i = i1++;
            const int on = 1 + 3 * i;
            if (const Op* Nop = ops.get({'N', i, 0})) {
                for (int x = 0; x < nb; ++x) {
                    const int mS = B.pm_S[x];
                    const int ds = S.md[mS], de = E.md[B.pm_E[x]];
                    const Sub* e1 = esub(x, 1);
                    const int64_t zo = phi;
                    bool any = false;
                    for (int o : S.msub[mS]) {
                        if (o < 0) continue;
                        g.begin();
                        bool got = false;
                        for (int i2 : S.msub[mS]) {
                            if (i2 < 0) continue;
                            for (int q : Nop->acting(i2, false)) {
                                const Blk& bk = Nop->blk[q];
                                if (bk.out != o) continue;
                                g.chunk(1.0, 1, bk.off, bk.cols, false, 0, B.poff[x] + (int64_t)S.sub[i2].off * de, de,
                                        false, S.sub[i2].dim);
                                got = true;
                            }
                        }
                        if (!got) continue;
                        const int64_t po = B.poff[x] + (int64_t)S.sub[o].off * de;
                        const int64_t zz = zo + (int64_t)S.sub[o].off * de;
                        g.end(2, zz, de, S.sub[o].dim, de, 0);
                        any = true;
                        seg(on, 1.0, 0, po, de, 2, zz, de, S.sub[o].dim, de);
                        if (e1) seg(on + 1, 1.0, 0, po + e1->off, de, 2, zz + e1->off, de, S.sub[o].dim, e1->dim);
                    }
                    if (any) phi += ((int64_t)ds * de + 31) / 32 * 32;
                }
            }
            const Op* C = delta_[i] == delta_[j] ? ops.get({'C', i, 0}) : nullptr;
            if (!C) continue;
            for (int x = 0; x < nb; ++x) {
                const Sub* e1 = esub(x, 1);
                if (!e1) continue;
                const int mS = B.pm_S[x];
                const int de = E.md[B.pm_E[x]];
                int m_out = -1;
                for (int i2 : S.msub[mS]) {
                    if (i2 < 0) continue;
                    for (int q : C->acting(i2, false)) m_out = S.sub[C->blk[q].out].m;
                }
                if (m_out < 0) continue;
                const int x2 = B.blk_of_S[m_out];
                const Sub* e0 = esub(x2, 0);
                if (!e0 || e0->base != e1->base) continue;
                const int de2 = E.md[B.pm_E[x2]];
                const int w = e1->dim;
                const double sign = (S.mq[mS].n() & 1) ? -1.0 : 1.0;
                const int64_t to = phi;
                bool any = false;
                for (int o : S.msub[m_out]) {
                    if (o < 0) continue;
                    g.begin();
                    bool got = false;
                    for (int i2 : S.msub[mS]) {
                        if (i2 < 0) continue;
                        for (int q : C->acting(i2, false)) {
                            const Blk& bk = C->blk[q];
                            if (bk.out != o) continue;
                            g.chunk(1.0, 1, bk.off, bk.cols, false, 0,
                                    B.poff[x] + (int64_t)S.sub[i2].off * de + e1->off, de, false, S.sub[i2].dim);
                            got = true;
                        }
                    }
                    if (!got) continue;
                    const int64_t tt = to + (int64_t)S.sub[o].off * w;
                    g.end(2, tt, w, S.sub[o].dim, w, 0);
                    any = true;
                    seg(on + 2, sign, 0, B.poff[x2] + (int64_t)S.sub[o].off * de2 + e0->off, de2, 2, tt, w,
                        S.sub[o].dim, w);
                }
                if (any) phi += ((int64_t)S.md[m_out] * w + 31) / 32 * 32;
            }
        }
        // bounds of every operand and output against its buffer (psi, ops, phi)
        const int64_t lim[3] = {psi_elems, ops.size, phi};
        auto inside = [&](int buf, int64_t off, int64_t rows, int64_t cols, int64_t ld) {
            return buf >= 0 && buf < 3 && off >= 0 && rows >= 1 && cols >= 1 && cols <= ld &&
                   off + (rows - 1) * ld + cols <= lim[buf];
        };
        for (const auto& ob : g.obs) {
            if (!inside(2, ob.coff, ob.M, ob.Nn, ob.ldc)) return fail(DMRG_ERR_DEVICE, "internal: measurement output out of range");
            for (int64_t c = ob.cb; c < ob.ce; ++c) {
                const GemmChunk& ch = g.chunks[c];
                if (!inside(ch.a_buf, ch.a_off, ob.M, ch.K, ch.lda) || !inside(ch.b_buf, ch.b_off, ch.K, ob.Nn, ch.ldb))
                    return fail(DMRG_ERR_DEVICE, "internal: measurement operand out of range");
            }
        }
        const int o0 = i0 == 0 ? 0 : 1 + 3 * i0, o1 = 1 + 3 * i1;
        std::vector<dmrgdev::SegDot> flat;
        std::vector<int32_t> obeg;
        for (int o = o0; o < o1; ++o) {
            obeg.push_back((int32_t)flat.size());
            for (const auto& sd : segs_of[o]) {
                if (!inside(sd.a_buf, sd.a_off, sd.rows, sd.cols, sd.lda) ||
                    !inside(sd.b_buf, sd.b_off, sd.rows, sd.cols, sd.ldb))
                    return fail(DMRG_ERR_DEVICE, "internal: measurement dot out of range");
                flat.push_back(sd);
            }
        }
        obeg.push_back((int32_t)flat.size());
        Buf phib, sb, obb, pb;
        TRY(alloc_buf(phib, std::max<int64_t>(phi, 1) * sizeof(double)));
        GemmPlan p;
        TRY(finish_plan(*this, g, p));
        BufTable bufs{psi_.p, ops.pool.p, phib.p};
        TRY(run_gemm(dmrgdev::P_F64, bufs, p));
        if (!flat.empty()) TRY(upload(sb, flat));
        TRY(upload(obb, obeg));
        TRY(alloc_buf(pb, std::max<size_t>(flat.size(), 1) * sizeof(double)));
        double* dbufs[3] = {psi_.d(), ops.pool.d(), phib.d()};
        DEV(dmrgdev::seg_dots(dev_, dbufs, flat.empty() ? nullptr : sb.as<dmrgdev::SegDot>(), (int)flat.size(),
                              obb.as<int32_t>(), o1 - o0, pb.d(), outb.d() + o0));
        DEV(dmrgdev::sync(dev_));
        i0 = i1;
    }
    std::vector<double> h(nout);
    DEV(dmrgdev::d2h(dev_, h.data(), outb.d(), (size_t)nout * sizeof(double)));
    const double nj = h[0];
    m_n1_[j] = nj;
    for (int i = 0; i <= b; ++i) {
        const size_t at = (size_t)i * N_ + j;
        m_pni_[at] = h[1 + 3 * i];
        m_pnj_[at] = nj;
        m_nn_[at] = h[2 + 3 * i];
        m_hop_[at] = h[3 + 3 * i];
    }
    if (b == 0) m_n1_[0] = h[1];
    return DMRG_OK;
}

dmrg_status Engine::orbital_entropies(double* s1, double* mutual, double* n1, double* nn, double* hop) {
    if (!meas_valid_) return fail(DMRG_ERR_STATE, "no completed sweep with measure = 1");
    const int n = N_;
    for (int p = 0; p < n; ++p) {
        const int a = order_[p];
        if (s1) s1[a] = entropy_one(m_n1_[p]);
        if (n1) n1[a] = m_n1_[p];
        if (mutual) mutual[(size_t)a * n + a] = 0.0;
        if (nn) nn[(size_t)a * n + a] = m_n1_[p];
        if (hop) hop[(size_t)a * n + a] = 0.0;
        for (int q = p + 1; q < n; ++q) {
            const int c = order_[q];
            const size_t at = (size_t)p * n + q;
            const double ni = m_pni_[at], nj = m_pnj_[at];
            if (mutual)
                mutual[(size_t)a * n + c] = mutual[(size_t)c * n + a] =
                    entropy_one(ni) + entropy_one(nj) - entropy_two(ni, nj, m_nn_[at], m_hop_[at]);
            if (nn) nn[(size_t)a * n + c] = nn[(size_t)c * n + a] = m_nn_[at];
            if (hop) hop[(size_t)a * n + c] = hop[(size_t)c * n + a] = m_hop_[at];
        }
    }
    return DMRG_OK;
}

// ========================================================== queries
dmrg_status Engine::layout(int32_t* bond, int64_t* dim, int32_t* nsec, int32_t* qn, int64_t* dims) {
    if (!cur_) return fail(DMRG_ERR_STATE, "no current bond (run a sweep first)");
    const Bond& B = *cur_;
    if (bond) *bond = B.b;
    if (dim) *dim = B.dim;
    if (nsec) *nsec = (int32_t)B.pm_S.size();
    for (size_t x = 0; x < B.pm_S.size(); ++x) {
        const QN& q = B.S.mq[B.pm_S[x]];
        if (qn) {
            qn[3 * x] = q.np;
            qn[3 * x + 1] = q.nn;
            qn[3 * x + 2] = q.tm;
        }
        if (dims) {
            dims[2 * x] = B.S.md[B.pm_S[x]];
            dims[2 * x + 1] = B.E.md[B.pm_E[x]];
        }
    }
    return DMRG_OK;
}

dmrg_status Engine::apply(const double* x, double* y, int prec) {
    if (!cur_) return fail(DMRG_ERR_STATE, "no current bond (run a sweep first)");
    if (!x || !y) return fail(DMRG_ERR_ARG, "null vector");
    if (prec < 0 || prec > 2) return fail(DMRG_ERR_ARG, "precision must be 0, 1 or 2");
    return heff_launch(*cur_, x, y, prec, false);
}

// y = H_eff x with every intermediate in the device's static scratch: the
// reduced-precision operator copies (converted here on every call), the
// reduced-precision x and y, Z and the split-K partial tiles.  No device
// memory is allocated or freed.  The launches are those of apply().
dmrg_status Engine::apply_static(const double* x, double* y, int prec) {
    if (!cur_) return fail(DMRG_ERR_STATE, "no current bond (run a sweep first)");
    if (!x || !y) return fail(DMRG_ERR_ARG, "null vector");
    if (prec < 0 || prec > 2) return fail(DMRG_ERR_ARG, "precision must be 0, 1 or 2");
    Bond& B = *cur_;
    size_t cap = 0;
    char* base = static_cast<char*>(dmrgdev::static_scratch(dev_, &cap));
    if (!base) return fail(DMRG_ERR_DEVICE, "static scratch is not available on this device");
    const bool low = prec != dmrgdev::P_F64;
    const size_t es = prec == dmrgdev::P_F64 ? 8 : (prec == dmrgdev::P_F32 ? 4 : 2);
    int64_t zmax = 0, slots = 0;
    for (auto& g : B.groups) {
        zmax = std::max(zmax, g.z_elems);
        slots = std::max({slots, g.p1.nslots, g.p2.nslots, g.p3.nslots});
    }
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t s_off = off;
    if (low) off += al((size_t)B.Sops.size * es);
    const size_t e_off = off;
    if (low) off += al((size_t)B.Eops.size * es);
    const size_t x_off = off;
    if (low) off += al((size_t)B.dim * es);
    const size_t y_off = off;
    if (low) off += al((size_t)B.dim * 4);
    const size_t z_off = off;
    off += al((size_t)std::max<int64_t>(zmax, 1) * es);
    const size_t p_off = off;
    off += al((size_t)slots * dmrgdev::kTileM * dmrgdev::kTileN * sizeof(double));
    off += 256;   // slack past the last operand, as for allocated blocks
    if (off > cap) {
        std::ostringstream m;
        m << "this bond needs " << off << " bytes of static scratch; the array holds " << cap
          << " (use dmrg_heff_apply)";
        return fail(DMRG_ERR_OUT_OF_MEMORY, m.str());
    }
    void* part = slots ? base + p_off : nullptr;
    if (!low) {
        for (auto& g : B.groups) {
            BufTable bufs{B.Sops.pool.p, B.Eops.pool.p, (void*)x, base + z_off, y};
            TRY(run_gemm(prec, bufs, g.p1, -1, dmrgdev::GK_HEFF_Z, part));
            TRY(run_gemm(prec, bufs, g.p2, -1, dmrgdev::GK_HEFF_Y, part));
            TRY(run_gemm(prec, bufs, g.p3, -1, dmrgdev::GK_OTHER, part));
        }
        return DMRG_OK;
    }
    DEV(dmrgdev::convert(dev_, dmrgdev::P_F64, B.Sops.pool.p, prec, base + s_off, B.Sops.size));
    DEV(dmrgdev::convert(dev_, dmrgdev::P_F64, B.Eops.pool.p, prec, base + e_off, B.Eops.size));
    DEV(dmrgdev::convert(dev_, dmrgdev::P_F64, x, prec, base + x_off, B.dim));
    for (auto& g : B.groups) {
        BufTable bufs{base + s_off, base + e_off, base + x_off, base + z_off, base + y_off};
        TRY(run_gemm(prec, bufs, g.p1, prec, dmrgdev::GK_HEFF_Z, part));
        TRY(run_gemm(prec, bufs, g.p2, dmrgdev::P_F32, dmrgdev::GK_HEFF_Y, part));
        TRY(run_gemm(prec, bufs, g.p3, dmrgdev::P_F32, dmrgdev::GK_OTHER, part));
    }
    DEV(dmrgdev::convert(dev_, dmrgdev::P_F32, base + y_off, dmrgdev::P_F64, y, B.dim));
    return DMRG_OK;
}

dmrg_status Engine::energy(double* E) {
    if (!E) return fail(DMRG_ERR_ARG, "null output");
    if (!have_energy_) return fail(DMRG_ERR_STATE, "no completed sweep");
    *E = energy_;
    return DMRG_OK;
}

dmrg_status Engine::get_psi(double* host) {
    if (!cur_ || !psi_.p) return fail(DMRG_ERR_STATE, "no state");
    if (!host) return fail(DMRG_ERR_ARG, "null output");
    DEV(dmrgdev::sync(dev_));
    DEV(dmrgdev::d2h(dev_, host, psi_.p, cur_->dim * sizeof(double)));
    return DMRG_OK;
}

dmrg_status Engine::configs(uint64_t* out) {
    if (!cur_) return fail(DMRG_ERR_STATE, "no current bond");
    const Bond& B = *cur_;
    const Stored& L = *L_[B.b];
    const Stored& R = *R_[B.b + 2];
    if (!L.has_cfg || !R.has_cfg) return fail(DMRG_ERR_STATE, "block bases are not determinant selections");
    for (size_t x = 0; x < B.pm_S.size(); ++x) {
        std::vector<uint64_t> sc, ec;
        for (int i : B.S.msub[B.pm_S[x]]) {
            if (i < 0) continue;
            for (uint64_t c : L.cfg[B.S.sub[i].base]) sc.push_back(c | (B.S.sub[i].sigma ? (1ull << B.S.site) : 0ull));
        }
        for (int j : B.E.msub[B.pm_E[x]]) {
            if (j < 0) continue;
            for (uint64_t c : R.cfg[B.E.sub[j].base]) ec.push_back(c | (B.E.sub[j].sigma ? (1ull << B.E.site) : 0ull));
        }
        int64_t o = B.poff[x];
        for (uint64_t a : sc)
            for (uint64_t c : ec) out[o++] = a | c;
    }
    return DMRG_OK;
}

}  // namespace dm
