// capi.cpp - extern "C" entry points of include/dmrg.h.  Argument checks,
// exception containment and status translation; the work is in engine.cpp.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <memory>
#include <thread>
#include <vector>

#include "../../include/dmrg.h"
#include "batch.h"
#include "device.h"
#include "engine.h"

struct dmrg_ctx {
    dmrgdev::Ctx* dev = nullptr;
    dm::Engine* eng = nullptr;
    std::string err;
};

namespace {
thread_local std::string g_create_err;

template <class F> dmrg_status guarded(dmrg_ctx* c, F&& f) {
    if (!c) return DMRG_ERR_ARG;
    try {
        dmrg_status s = f();
        c->err = s == DMRG_OK ? std::string() : c->eng->error();
        return s;
    } catch (const std::bad_alloc&) {
        c->err = "host allocation failed";
        return DMRG_ERR_OUT_OF_MEMORY;
    } catch (const std::exception& e) {
        c->err = e.what();
        return DMRG_ERR_DEVICE;
    } catch (...) {
        c->err = "unknown exception";
        return DMRG_ERR_DEVICE;
    }
}
}  // namespace

extern "C" {

void dmrg_default_options(dmrg_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = DMRG_FP64;
    o->seed = 1507;
    o->davidson_tol = 1e-7;
    o->davidson_max_iter = 100;
    o->davidson_max_subspace = 24;
    o->noise = 0.0;
    o->noise_sweeps = 0;
    o->select_basis = 0;
    o->tie_tol = 1e-13;
    o->device = 0;
    o->stream = nullptr;
    o->mem_cap_bytes = 0;
    o->scratch_bytes = 0;
    o->trunc_eps = 0.0;
    o->d_min = 0;
    o->n_states = 1;
    o->measure = 0;
    o->graph = 0;
    o->group_products = 1;
}

dmrg_status dmrg_create(const dmrg_options* opt, dmrg_ctx** out) {
    if (!out) return DMRG_ERR_ARG;
    *out = nullptr;
    dmrg_options o;
    dmrg_default_options(&o);
    if (opt) o = *opt;
    if (o.precision < 0 || o.precision > 2 || o.davidson_tol <= 0 || o.davidson_max_iter < 1 ||
        o.davidson_max_subspace < 2 || o.davidson_max_subspace > 32 || o.noise < 0 || o.tie_tol < 0 ||
        !(o.trunc_eps >= 0) || o.d_min < 0 || o.n_states < 1 || o.n_states > 2 ||
        (o.measure != 0 && o.measure != 1) || (o.graph != 0 && o.graph != 1) ||
        (o.group_products != 0 && o.group_products != 1)) {
        g_create_err = "invalid option value";
        return DMRG_ERR_ARG;
    }
    try {
        auto* c = new dmrg_ctx();
        char buf[512] = {0};
        if (dmrgdev::ctx_create(o.device, o.stream, &c->dev, buf, sizeof(buf))) {
            g_create_err = buf;
            delete c;
            return DMRG_ERR_DEVICE;
        }
        c->eng = new dm::Engine(c->dev, o);
        *out = c;
        return DMRG_OK;
    } catch (...) {
        g_create_err = "allocation failed";
        return DMRG_ERR_OUT_OF_MEMORY;
    }
}

void dmrg_destroy(dmrg_ctx* c) {
    if (!c) return;
    delete c->eng;
    dmrgdev::ctx_destroy(c->dev);
    delete c;
}

dmrg_status dmrg_load_hamiltonian(dmrg_ctx* c, int32_t n, const int32_t* species, const int32_t* two_m,
                                  const double* eps, const double* V, int32_t n_p, int32_t n_n,
                                  int32_t two_M) {
    return guarded(c, [&] { return c->eng->load(n, species, two_m, eps, V, n_p, n_n, two_M); });
}

dmrg_status dmrg_sweep(dmrg_ctx* c, const int32_t* ordering, int32_t D, dmrg_sweep_stats* out) {
    return guarded(c, [&] { return c->eng->steps(ordering, D, INT64_MAX, true, out); });
}

dmrg_status dmrg_sweep_steps(dmrg_ctx* c, const int32_t* ordering, int32_t D, int32_t n_steps,
                             dmrg_sweep_stats* out) {
    if (n_steps < 0) return DMRG_ERR_ARG;
    return guarded(c, [&] { return c->eng->steps(ordering, D, n_steps, false, out); });
}

dmrg_status dmrg_heff_layout(dmrg_ctx* c, int32_t* bond, int64_t* dim, int32_t* n_sectors,
                             int32_t* sector_qn, int64_t* sector_dims) {
    return guarded(c, [&] { return c->eng->layout(bond, dim, n_sectors, sector_qn, sector_dims); });
}

dmrg_status dmrg_heff_apply(dmrg_ctx* c, const double* x, double* y, int32_t precision) {
    return guarded(c, [&] { return c->eng->apply(x, y, precision); });
}

dmrg_status dmrg_heff_apply_noalloc(dmrg_ctx* c, const double* x, double* y, int32_t precision) {
    return guarded(c, [&] { return c->eng->apply_static(x, y, precision); });
}

dmrg_status dmrg_set_cideas(dmrg_ctx* c, const double* s1, const double* n1) {
    return guarded(c, [&] { return c->eng->set_cideas(s1, n1); });
}

dmrg_status dmrg_check_fp64(dmrg_ctx* c, int32_t on) {
    if (!c) return DMRG_ERR_ARG;
    if (on != 0 && on != 1) {
        c->err = "on must be 0 or 1";
        return DMRG_ERR_ARG;
    }
    return guarded(c, [&] { return c->eng->set_check_fp64(on != 0); });
}

dmrg_status dmrg_energy(dmrg_ctx* c, double* E) {
    return guarded(c, [&] { return c->eng->energy(E); });
}

dmrg_status dmrg_get_psi(dmrg_ctx* c, double* psi) {
    return guarded(c, [&] { return c->eng->get_psi(psi); });
}

dmrg_status dmrg_orbital_entropies(dmrg_ctx* c, double* s1, double* mutual, double* n1, double* nn, double* hop) {
    return guarded(c, [&] { return c->eng->orbital_entropies(s1, mutual, n1, nn, hop); });
}

dmrg_status dmrg_fiedler_ordering(const double* mutual, int32_t n, int32_t* ordering, double* fiedler_value) {
    if (!mutual || !ordering || n < 1) return DMRG_ERR_ARG;
    try {
        return dm::fiedler_ordering(mutual, n, ordering, fiedler_value) ? DMRG_OK : DMRG_ERR_ARG;
    } catch (...) {
        return DMRG_ERR_ARG;
    }
}

dmrg_status dmrg_heff_configs(dmrg_ctx* c, uint64_t* configs) {
    if (!configs) return DMRG_ERR_ARG;
    return guarded(c, [&] { return c->eng->configs(configs); });
}

dmrg_status dmrg_sweep_many(dmrg_ctx** ctxs, int32_t n, const int32_t* const* orderings, const int32_t* D,
                            dmrg_sweep_stats* out) {
    if (!ctxs || n < 0 || !D) return DMRG_ERR_ARG;
    for (int32_t i = 0; i < n; ++i) {
        if (!ctxs[i]) return DMRG_ERR_ARG;
        for (int32_t j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return DMRG_ERR_ARG;   // a context runs on one thread at a time
    }
    // Every context is driven by a host thread of its own (at most 16 at a
    // time).  When all of them run on one device and ask for grouped
    // products, their H_eff products go through one batch: products pending together are launched as one
    // grouped GEMM per phase over all their plans.  Each context's work keeps
    // its own order, so the results equal one-at-a-time sweeps.
    std::vector<dmrg_status> st(n, DMRG_OK);
    std::vector<dmrg_sweep_stats> res(n);
    std::atomic<int32_t> next(0);
    // Host threads: the planning of a context is CPU work, so more threads
    // than the host can run only add contention (and waiting threads spin
    // in the HIP runtime's synchronisations).
    const int nt = (int)std::min<int32_t>(n, 16);
    std::unique_ptr<dm::Batch> batch;
    bool same = n > 1;
    for (int32_t i = 0; i < n && same; ++i) same = ctxs[i]->eng->options().group_products == 1;
    for (int32_t i = 1; i < n && same; ++i)
        same = dmrgdev::ctx_device(ctxs[i]->dev) == dmrgdev::ctx_device(ctxs[0]->dev);
    if (same) {
        batch.reset(new dm::Batch(dmrgdev::ctx_device(ctxs[0]->dev)));
        if (!batch->ok()) batch.reset();   // independent sweeps
    }
    for (int32_t i = 0; i < n; ++i) {
        ctxs[i]->eng->set_in_many(true);
        if (batch) ctxs[i]->eng->attach_batch(batch.get());
    }
    auto worker = [&] {
        for (int32_t i = next++; i < n; i = next++) {
            dmrgdev::bind(ctxs[i]->dev);
            dmrg_sweep_stats s{};
            st[i] = dmrg_sweep(ctxs[i], orderings ? orderings[i] : nullptr, D[i], &s);
            s.status = st[i];
            res[i] = s;
        }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
    worker();
    for (auto& t : pool) t.join();
    for (int32_t i = 0; i < n; ++i) {
        ctxs[i]->eng->set_in_many(false);
        if (batch) ctxs[i]->eng->attach_batch(nullptr);
    }
    dmrg_status worst = DMRG_OK;
    for (int32_t i = 0; i < n; ++i) {
        if (out) out[i] = res[i];
        const dmrg_status s = st[i];
        if (s < 0 && worst >= 0) worst = s;
        else if (s > worst && worst >= 0) worst = s;
    }
    return worst;
}

const char* dmrg_status_string(dmrg_status s) {
    switch (s) {
        case DMRG_OK: return "ok";
        case DMRG_WARN_NOT_CONVERGED: return "Davidson did not converge";
        case DMRG_ERR_ARG: return "invalid argument";
        case DMRG_ERR_HAMILTONIAN: return "invalid Hamiltonian";
        case DMRG_ERR_TARGET: return "unreachable target";
        case DMRG_ERR_STATE: return "invalid state for this call";
        case DMRG_ERR_OUT_OF_MEMORY: return "out of memory";
        case DMRG_ERR_DEVICE: return "device error";
    }
    return "unknown status";
}

const char* dmrg_last_error(const dmrg_ctx* c) {
    if (!c) return g_create_err.c_str();
    return c->err.c_str();
}

}  // extern "C"
