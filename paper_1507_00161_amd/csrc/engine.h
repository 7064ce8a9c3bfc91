// engine.h - host side of the two-site DMRG: quantum-number bookkeeping,
// block-operator catalogue and blocking recipes, work lists for the device
// kernels, and the sweep / Davidson / truncation control.
#pragma once
#include <algorithm>
#include <array>
#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/dmrg.h"
#include "device.h"

namespace dm {

struct QN {
    int np = 0, nn = 0, tm = 0;
    QN() = default;
    QN(int a, int b, int c) : np(a), nn(b), tm(c) {}
    bool operator<(const QN& o) const {
        if (np != o.np) return np < o.np;
        if (nn != o.nn) return nn < o.nn;
        return tm < o.tm;
    }
    bool operator==(const QN& o) const { return np == o.np && nn == o.nn && tm == o.tm; }
    bool operator!=(const QN& o) const { return !(*this == o); }
    QN operator+(const QN& o) const { return {np + o.np, nn + o.nn, tm + o.tm}; }
    QN operator-(const QN& o) const { return {np - o.np, nn - o.nn, tm - o.tm}; }
    QN operator-() const { return {-np, -nn, -tm}; }
    int n() const { return np + nn; }
};

// operator catalogue key: H; C i (c+_i); R i; A i j; B i j; P i j; Q i j
struct Key {
    char k;
    int i, j;
    bool operator<(const Key& o) const {
        if (k != o.k) return k < o.k;
        if (i != o.i) return i < o.i;
        return j < o.j;
    }
};

class Engine;

// owning device allocation, counted against the context's memory cap
struct Buf {
    Engine* eng = nullptr;
    void* p = nullptr;
    size_t bytes = 0;
    Buf() = default;
    Buf(const Buf&) = delete;
    Buf& operator=(const Buf&) = delete;
    Buf(Buf&& o) noexcept { *this = std::move(o); }
    Buf& operator=(Buf&& o) noexcept;
    ~Buf() { reset(); }
    void reset();
    double* d() const { return static_cast<double*>(p); }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

struct Basis {
    std::vector<QN> q;
    std::vector<int> d;
    std::map<QN, int> idx;
    int find(const QN& x) const {
        auto it = idx.find(x);
        return it == idx.end() ? -1 : it->second;
    }
    void add(const QN& x, int dim) {
        idx[x] = (int)q.size();
        q.push_back(x);
        d.push_back(dim);
    }
    int64_t total() const {
        int64_t t = 0;
        for (int x : d) t += x;
        return t;
    }
};

// Enlarged block S = L*s or E = s*R.  Its states are grouped in sub-sectors
// (base sector, site occupation sigma); sub-sectors with equal quantum
// numbers form a merged sector whose rows list sigma = 0 first.
struct Sub {
    int m, base, sigma, off, dim;
    QN q;
};
struct Enl {
    char side = 'L';
    int site = 0;
    QN dsite;
    std::vector<QN> mq;
    std::vector<int> md;
    std::vector<Sub> sub;
    std::vector<std::array<int, 2>> msub;       // merged -> sub index per sigma (-1: absent)
    std::map<std::pair<int, int>, int> sub_of;  // (base sector, sigma) -> sub index
    std::vector<int> sub_tab;                   // the same as a table at 2 base + sigma
    std::map<QN, int> midx;
    int find_m(const QN& x) const {
        auto it = midx.find(x);
        return it == midx.end() ? -1 : it->second;
    }
    int find_sub(int base, int sigma) const {
        const size_t i = 2 * (size_t)base + sigma;
        return base >= 0 && i < sub_tab.size() ? sub_tab[i] : -1;
    }
};

struct Blk {
    int out, in;
    int64_t off;
    int rows, cols;
};
// Block-sparse operator with one quantum-number shift dq.  On a stored block
// (merged sectors) an input sector has at most one block; on an enlarged block
// (sub-sectors) it can have two, whose site occupations differ.
struct Op {
    QN dq;
    int par = 0;
    std::vector<Blk> blk;
    std::unordered_map<int, std::vector<int>> by_in, by_out;
    const std::vector<int>& ins(int s) const {
        static const std::vector<int> none;
        auto it = by_in.find(s);
        return it == by_in.end() ? none : it->second;
    }
    const std::vector<int>& outs(int s) const {
        static const std::vector<int> none;
        auto it = by_out.find(s);
        return it == by_out.end() ? none : it->second;
    }
    // the single block on an input (output) sector of a stored block
    const Blk* in_blk(int s) const {
        auto& v = ins(s);
        return v.empty() ? nullptr : &blk[v[0]];
    }
    const Blk* out_blk(int s) const {
        auto& v = outs(s);
        return v.empty() ? nullptr : &blk[v[0]];
    }
    // blocks acting on sector s of op (trans = 0) or of op^T (trans = 1)
    const std::vector<int>& acting(int s, bool trans) const { return trans ? outs(s) : ins(s); }
    void index() {
        by_in.clear();
        by_out.clear();
        for (size_t x = 0; x < blk.size(); ++x) {
            by_in[blk[x].in].push_back((int)x);
            by_out[blk[x].out].push_back((int)x);
        }
    }
};

struct OpSet {
    std::map<Key, int> idx;
    std::vector<Op> ops;
    std::vector<Key> keys;
    Buf pool;               // FP64 blocks
    Buf pool_lo;            // reduced-precision copy (mixed modes)
    int lo_prec = -1;
    int64_t size = 0;       // elements
    const Op* get(const Key& k) const {
        auto it = idx.find(k);
        return it == idx.end() ? nullptr : &ops[it->second];
    }
    int find(const Key& k) const {
        auto it = idx.find(k);
        return it == idx.end() ? -1 : it->second;
    }
    int add(const Key& k, Op&& op) {
        int x = (int)ops.size();
        idx[k] = x;
        keys.push_back(k);
        ops.push_back(std::move(op));
        return x;
    }
    int64_t alloc_block(int rows, int cols) {
        int64_t off = size;
        size += ((int64_t)rows * cols + 31) / 32 * 32;
        return off;
    }
};

// stored (renormalised) left block L = sites [0, hi) or right block R = sites [lo, N)
struct Stored {
    char side = 'L';
    int lo = 0, hi = 0;
    bool normal = true;            // normal (A, B) rather than complementary (P, Q) pair ops
    Basis basis;
    OpSet ops;
    // isometry that created the block from its composite (for prediction):
    // kept sector x <- composite merged sector comp_m[x], comp_dim x kept, row-major
    Enl comp;
    std::vector<int> comp_m;
    std::vector<int64_t> iso_off;
    Buf iso;
    bool has_cfg = false;
    std::vector<std::vector<uint64_t>> cfg;   // determinant per state (chain-position bits)
    int length() const { return hi - lo; }
};

// one term of H_eff: y += coef * sign * op(A) psi op(B)^T, sign = (-1)^{par n(S sector)}
// taken on the input S sector (sign_out = 0) or the output one (sign_out = 1)
struct Term {
    double coef;
    int a, b;          // op index in S / E op sets, -1 = identity
    bool ta, tb;
    bool sign_out;
    int par;
};

using BufTable = std::array<void*, dmrgdev::kMaxBufs>;

struct GemmPlan {
    // task, chunk, reduction and schedule lists: one device allocation, one upload
    Buf dev;
    dmrgdev::GemmTask* tasks = nullptr;
    dmrgdev::GemmChunk* chunks = nullptr;
    dmrgdev::RedTask* reds = nullptr;
    int32_t* wg_off = nullptr;
    int ntasks = 0, nreds = 0;
    int nwg = 0, nfull = 0;   // persistent work-groups; tasks with chunks
    int64_t nslots = 0;     // split-K partial tiles
    int64_t nchunks = 0;
    double flops = 0.0;    // useful: 2 M N K per chunk over the columns that can be nonzero
    double issued = 0.0;   // 2 M N K per chunk over the whole output block width
    double elems = 0.0;    // operand elements read + result elements written (algorithmic)
};

struct HeffGroup {
    GemmPlan p1, p2;    // Z = psi op(B)^T ; y (+)= op(A) Z over full-width row blocks
    GemmPlan p3;        // y += psi op(B)^T of the E-only term, into sub-blocks
    int64_t z_elems = 0;
};

struct Bond {
    int b = 0;
    int64_t gen = 0;      // distinct for every bond set up by a context
    Enl S, E;
    OpSet Sops, Eops;
    // psi layout: merged S sector pm_S[x] with E sector pm_E[x], offset poff[x]
    std::vector<int> pm_S, pm_E;
    std::vector<int64_t> poff;
    std::vector<int> blk_of_S;     // S merged -> psi block (-1)
    int64_t dim = 0;
    std::vector<Term> terms;
    std::vector<HeffGroup> groups;
    double flops = 0.0;       // useful flops of the launches of one product
    double flops_alg = 0.0;   // algorithmic flops of one product (cheaper contraction order)
    Buf diag;
    int lo_prec = -1;
};

struct LB;   // linear-combination task builder (engine.cpp)
class Batch;  // products of several contexts launched together (batch.h)

class Engine {
public:
    const dmrg_options& options() const { return opt_; }
    // host threads for a planning loop of n independent items: at most 16 (the
    // host's share), 1 while dmrg_sweep_many runs contexts side by side
    int host_threads(int64_t n) const {
        if (in_many_ || n < 64) return 1;
        const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        return (int)std::min<int64_t>(n / 32, std::min(16u, hw));
    }
    Engine(dmrgdev::Ctx* dev, const dmrg_options& opt) : dev_(dev), opt_(opt) {}
    ~Engine();

    dmrg_status load(int n, const int32_t* species, const int32_t* two_m, const double* eps,
                     const double* V, int n_p, int n_n, int two_M);
    dmrg_status steps(const int32_t* ordering, int D, int64_t max_steps, bool until_sweep_end,
                      dmrg_sweep_stats* st);
    dmrg_status layout(int32_t* bond, int64_t* dim, int32_t* nsec, int32_t* qn, int64_t* dims);
    dmrg_status apply(const double* x, double* y, int prec);
    dmrg_status apply_static(const double* x, double* y, int prec);
    dmrg_status energy(double* E);
    dmrg_status get_psi(double* host);
    dmrg_status configs(uint64_t* out);
    dmrg_status orbital_entropies(double* s1, double* mutual, double* n1, double* nn, double* hop);
    bool measuring() const { return opt_.measure != 0; }
    dmrg_status set_cideas(const double* s1, const double* n1);
    // while set, H_eff products of single-group bonds go through the batch
    void attach_batch(Batch* b) { batch_ = b; }
    // set while dmrg_sweep_many drives this context: its products are then
    // launched directly (or in groups), never as captured graphs
    void set_in_many(bool on) { in_many_ = on; }
    dmrg_status set_check_fp64(bool on) {
        check_fp64_ = on;
        return DMRG_OK;
    }

    const std::string& error() const { return err_; }
    dmrg_status fail(dmrg_status s, const std::string& msg) {
        err_ = msg;
        return s;
    }
    void* dalloc(size_t bytes);
    void dfree(void* p, size_t bytes);
    dmrgdev::Ctx* dev() const { return dev_; }

    // used by the plan builders
    double V(int i, int j, int k, int l) const {
        return V_[(((size_t)i * N_ + j) * N_ + k) * N_ + l];
    }
    int N() const { return N_; }
    const QN& delta(int i) const { return delta_[i]; }
    double eps(int i) const { return eps_[i]; }
    bool normal_S(int b) const { return b + 1 <= N_ - b - 1; }
    bool left_normal(int len) const { return normal_S(len); }
    bool right_normal(int lo) const { return N_ - lo + 1 < lo - 1; }
    template <class T> dmrg_status upload(Buf& b, const std::vector<T>& v);
    dmrg_status alloc_buf(Buf& b, size_t bytes);

private:
    dmrgdev::Ctx* dev_;
    bool in_many_ = false;
    dmrg_options opt_;
    std::string err_;
    int N_ = 0;
    std::vector<int> sp0_, tm0_;
    std::vector<double> eps0_, V0_;
    std::vector<int> order_;
    std::vector<double> eps_, V_;
    std::vector<QN> delta_;
    QN T_;
    bool loaded_ = false;
    // per-species subset sums of 2m: ok[k][tm + off] for k particles
    struct Reach {
        int off = 0, width = 0;
        std::vector<std::vector<char>> p, n;
    };
    std::vector<Reach> pre_;     // pre_[b]: sites 0..b-1
    // Stream-ordered device memory cache.  Every kernel and copy of a context
    // runs on its one stream, so a freed block can be handed out again at once:
    // later users are ordered after earlier ones.  This keeps hipFree (which
    // waits for the device) out of the sweep.  Declared before every Buf so
    // that it outlives them.
    size_t mem_used_ = 0;        // live + cached bytes
    size_t cached_ = 0;
    bool dying_ = false;
    std::multimap<size_t, void*> cache_;
    std::unordered_map<void*, size_t> live_;
    void trim_cache(size_t keep);

    // DMRG state
    bool init_ = false;
    int sweeps_done_ = 0;
    int dir_ = 0, bond_ = 0;     // position in the sweep schedule
    bool fresh_ = false;
    std::vector<std::unique_ptr<Stored>> L_, R_;
    std::unique_ptr<Bond> cur_;
    Buf psi_;
    Buf psi1_;                  // the second state (n_states = 2)
    double theta_ = 0.0;
    bool have_energy_ = false;
    double energy_ = 0.0;
    double prev_sweep_energy_ = 0.0;   // energy of the last full sweep since the blocks were set up
    bool have_prev_sweep_ = false;
    double sweep_min_ = 0.0;
    double sweep_min1_ = 0.0;   // second state
    double theta1_ = 0.0;
    int sweep_steps_ = 0;
    dmrg_sweep_stats acc_{};
    // Davidson workspace
    Buf dv_V_, dv_W_, dv_x_, dv_hx_, dv_r_, dv_t_, dv_small_;
    int64_t dv_cap_ = 0;
    // scratch
    Buf z_, xlo_, ylo_, scr_a_, scr_b_, scal_;
    double heff_time_ = 0.0;   // device seconds of H_eff products in the current solve
    bool check_fp64_ = false;  // repeat mixed solves in FP64 (diagnostic)
    Batch* batch_ = nullptr;
    void* ev_ready_ = nullptr;  // product input ready (context stream)
    void* ev_done_ = nullptr;   // product launched (batch stream)
    dmrg_status heff_batched(Bond& B, const double* x, double* y, int prec);
    // HIP graph of the current bond's product (option graph)
    int64_t bond_gen_ = 0;
    void* graph_exec_ = nullptr;
    int64_t graph_gen_ = -1;
    int graph_prec_ = -1;
    Buf gin_, gout_;
    dmrg_status heff_graph(Bond& B, const double* x, double* y, int prec);
    dmrg_status heff_direct(Bond& B, const double* x, double* y, int prec, bool timed);
    bool force_fp64_ = false;  // the solve in progress uses FP64 products only
    Buf chk_psi_;              // guess kept for the repeat

    bool reachable(const Reach& r, const QN& q) const;
    Reach make_reach(int a, int b) const;

    dmrg_status set_order(const int32_t* ordering);
    dmrg_status initialize(int D);
    std::unique_ptr<Stored> vacuum(char side, int lo);
    bool enlarge_plan(const Stored& base, char side, const std::vector<QN>& allowed, Enl& en, OpSet& ops,
                      LB& lb, std::string& why) const;
    dmrg_status enlarge_run(const Stored& base, OpSet& ops, LB& lb);
    dmrg_status enlarge(const Stored& base, char side, const std::vector<QN>& allowed,
                        Enl& en, OpSet& ops);
    dmrg_status renormalize(const Enl& en, const OpSet& ops, bool normal_in, Stored& out,
                            const std::vector<int>& keep_m, const std::vector<int>& kdim);
    dmrg_status setup_bond(int b, std::unique_ptr<Bond>& out);
    dmrg_status build_heff_plan(Bond& B);
    dmrg_status build_diag(Bond& B);
    dmrg_status heff(Bond& B, const double* x, double* y, int prec);
    dmrg_status heff_launch(Bond& B, const double* x, double* y, int prec, bool timed);
    void account(const HeffGroup& g, double es1, double es2);
    dmrg_status ensure_lo(Bond& B, int prec);
    dmrg_status davidson(Bond& B, Buf& psi, const double* lock, double* theta, int64_t* nlo, int64_t* n64,
                         bool* conv);
    dmrg_status truncate_and_move(int D, double alpha, double* disc);
    dmrg_status density_matrix(Bond& B, const Buf& psi, double weight, int beta, bool left, double alpha, Buf& rho,
                               const std::vector<int64_t>& roff, const std::vector<int>& rld);
    dmrg_status random_psi(Bond& B, Buf& out);
    // ev_start / ev_stop >= 0: those events are recorded at the GEMM kernel's own
    // start and end (both at once when the plan has no tasks); partials: split-K
    // partial tiles supplied by the caller (else the engine's own buffer)
    dmrg_status run_gemm(int prec, BufTable bufs, const GemmPlan& p, int cprec = -1,
                         int kind = dmrgdev::GK_OTHER, void* partials = nullptr, int ev_start = -1,
                         int ev_stop = -1);
    dmrg_status ensure_partials(int64_t slots);
    Buf partial_;
    dmrg_status ensure_dv(int64_t n, int kmax);
    // orbital correlations of the current sweep's right-to-left half, in chain
    // positions: n1[p]; for p < q (at p * N + q) the pair's <n_p>, <n_q>,
    // <n_p n_q> and <c+_p c_q>, all from the state at bond q - 1
    dmrg_status measure_bond(Bond& B);
    void reset_measure();
    std::vector<double> m_n1_, m_pni_, m_pnj_, m_nn_, m_hop_;
    bool meas_valid_ = false;
    // CI-DEAS start: profile in site indices, in chain positions, reference determinant
    bool cideas_ = false;
    std::vector<double> cds_site_, cdn_site_, cd_s_;
    uint64_t cd_ref_ = 0;
    void cideas_chain();
    std::vector<std::vector<double>> cideas_iso(const Enl& comp, const Stored& base, int D, int lo,
                                                std::vector<int>& kept, std::vector<std::vector<int>>& chosen);
    std::vector<std::vector<double>> selection_iso(const std::vector<int>& dims, int D, int tag,
                                                   int pos, const std::vector<QN>& qs, bool mix,
                                                   std::vector<int>& kept,
                                                   std::vector<std::vector<int>>* chosen);
};

// entropy.cpp: entropies of rho_i and rho_ij from the correlations, and the
// Fiedler-vector ordering of a mutual-information matrix (false: bad input)
double entropy_one(double n_i);
double entropy_two(double n_i, double n_j, double nn_ij, double hop_ij);
bool fiedler_ordering(const double* mutual, int n, int32_t* ordering, double* fiedler_value);

}  // namespace dm
