// C-ABI entry points of libstokestree (declared in include/stokestree.h).  Validates
// arguments, converts internal errors to status codes and keeps a thread-local
// message for stk_last_error().
#include <cmath>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "stk_internal.hpp"
#include "stk_math.hpp"

struct stk_tree {
    stk::Tree t;
};
struct stk_plan {
    stk::Plan p;
};

namespace {

thread_local std::string g_err;

template <class F> stk_status guarded(F &&f) {
    try {
        f();
        g_err.clear();
        return STK_OK;
    } catch (const stk::Error &e) {
        g_err = e.what();
        return e.status;
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        return STK_ENOMEM;
    } catch (const std::exception &e) {
        g_err = e.what();
        return STK_EDEVICE;
    } catch (...) {
        g_err = "unknown error";
        return STK_EDEVICE;
    }
}

inline hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

void check_device(int dev) {
    int cur = -1;
    STK_HIP(hipGetDevice(&cur));
    stk::require(cur == dev, "handle used on a device other than the one it was created on");
}

void check_common(const double *pts, int64_t n, const char *what) {
    stk::require(pts != nullptr, std::string(what) + " is NULL");
    stk::require(n >= 1, std::string(what) + ": count must be >= 1");
    stk::require(n < (int64_t(1) << 31) / 8, std::string(what) + ": count too large (int32 indexing)");
}

// Two more streams per device (default priority; created on first use, kept until the
// process exits): on the first stk_evaluate computes the moments while the caller's stream
// sorts the targets and builds the interaction lists, on the second it builds the sparse
// far entries' cluster-major view while the caller's stream builds the near field's.
hipStream_t side_stream(int dev, int which = 0) {
    static std::mutex mu;
    static std::vector<hipStream_t> *streams = new std::vector<hipStream_t>();
    std::lock_guard<std::mutex> lk(mu);
    const size_t k = 2 * size_t(dev) + size_t(which);
    if (k >= streams->size()) streams->resize(k + 1, nullptr);
    hipStream_t &sd = (*streams)[k];
    if (!sd) STK_HIP(hipStreamCreateWithFlags(&sd, hipStreamNonBlocking));
    return sd;
}

// Tree on the caller's stream, then the moments on the side stream (after the tree and
// everything queued before it) while the evaluation proceeds; the evaluation waits for
// the source records before its near field and for the moments before its far field.
void tree_moments_evaluate(stk::Tree &tree, stk::Plan &pl, const double *targets, int64_t m, const double *sources,
                           int64_t n, const double *f, const double *h, const double *nu, int32_t k_rhs, int32_t p,
                           double theta, int32_t n0, stk_precision prec, double *u_out, bool same, hipStream_t s) {
    stk::build_tree(tree, sources, n, n0, s);
    hipStream_t s2 = side_stream(tree.device);
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // tree built, records written, moments done
    for (hipEvent_t &e : ev) STK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    try {
        STK_HIP(hipEventRecord(ev[0], s));
        STK_HIP(hipStreamWaitEvent(s2, ev[0], 0));
        stk::compute_moments(tree, f, h, nu, k_rhs, p, prec, s2, ev[1]);
        STK_HIP(hipEventRecord(ev[2], s2));
        pl.records_ready = ev[1];
        pl.moments_ready = ev[2];
        pl.aux = side_stream(tree.device, 1);
        stk::evaluate(tree, pl, targets, m, theta, u_out, same, s);
    } catch (...) {
        pl.records_ready = pl.moments_ready = nullptr;
        (void)hipStreamSynchronize(s2);
        if (pl.aux) (void)hipStreamSynchronize(pl.aux);
        pl.aux = nullptr;
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        throw;
    }
    pl.records_ready = pl.moments_ready = nullptr;
    pl.aux = nullptr;
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}

// Plans that own their tree, parked by stk_plan_destroy for the next stk_evaluate with
// keep_plan on the same device: their buffers keep their capacity, so a loop of
// forward + adjoint calls allocates and frees no device memory after the first pass
// (hipFree synchronises the device on every call).  The pool is never destroyed: parked
// device memory returns to the system when the process exits or stk_plan_cache_clear
// runs.
constexpr size_t PLAN_POOL_PER_DEVICE = 2;

struct PlanPool {
    std::mutex mu;
    std::vector<stk_plan *> parked;
};

PlanPool &plan_pool() {
    static PlanPool *pool = new PlanPool();
    return *pool;
}

stk_plan *take_plan(int dev) {
    PlanPool &pp = plan_pool();
    std::lock_guard<std::mutex> lk(pp.mu);
    for (size_t i = 0; i < pp.parked.size(); ++i) {
        stk_plan *pl = pp.parked[i];
        if (pl->p.tree->device == dev) {
            pp.parked.erase(pp.parked.begin() + i);
            pl->p.forced = false;
            return pl;
        }
    }
    return nullptr;
}

// Park a plan with an owned tree when its device has room, after the device has finished
// all work queued so far (the plan's kernels may still be in flight on any stream);
// otherwise delete it.
void park_or_delete(stk_plan *pl) {
    if (!pl->p.owns_tree || pl->p.tree == nullptr) {
        delete pl;
        return;
    }
    const int dev = pl->p.tree->device;
    PlanPool &pp = plan_pool();
    {
        std::lock_guard<std::mutex> lk(pp.mu);
        size_t here = 0;
        for (stk_plan *q : pp.parked) here += q->p.tree->device == dev;
        if (here >= PLAN_POOL_PER_DEVICE) {
            delete pl;
            return;
        }
    }
    int cur = -1;
    bool ok = hipGetDevice(&cur) == hipSuccess;
    if (ok && cur != dev) ok = hipSetDevice(dev) == hipSuccess;
    if (ok) ok = hipDeviceSynchronize() == hipSuccess;
    if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
    if (!ok) {
        delete pl;
        return;
    }
    std::lock_guard<std::mutex> lk(pp.mu);
    pp.parked.push_back(pl);
}

}  // namespace

extern "C" {

const char *stk_last_error(void) { return g_err.c_str(); }

stk_status stk_build_tree(const double *src, int64_t n, int32_t n0, void *stream, stk_tree **out) {
    return guarded([&] {
        check_common(src, n, "sources");
        stk::require(out != nullptr, "out is NULL");
        stk::require(n0 >= 1, "n0 must be >= 1");
        *out = nullptr;
        auto *h = new stk_tree();
        try {
            STK_HIP(hipGetDevice(&h->t.device));
            stk::build_tree(h->t, src, n, n0, as_stream(stream));
            STK_HIP(hipStreamSynchronize(as_stream(stream)));
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
    });
}

stk_status stk_compute_moments(stk_tree *t, const double *f, const double *h, const double *nu, int32_t k_rhs,
                               int32_t p, stk_precision prec, void *stream) {
    return guarded([&] {
        stk::require(t != nullptr, "tree is NULL");
        stk::require(f && h && nu, "f, h and nu must be non-NULL");
        stk::require(k_rhs >= 1 && k_rhs <= 64, "k_rhs must be in [1, 64]");
        stk::require(p >= 0 && p <= STK_P_MAX, "p must be in [0, STK_P_MAX]");
        stk::require(prec == STK_FP64 || prec == STK_MIXED, "unknown precision");
        check_device(t->t.device);
        stk::compute_moments(t->t, f, h, nu, k_rhs, p, prec, as_stream(stream));
    });
}

stk_status stk_evaluate_tree(stk_tree *t, const double *targets, int64_t m, double theta, double *u_out,
                             stk_plan **keep_plan, void *stream) {
    return guarded([&] {
        stk::require(t != nullptr, "tree is NULL");
        check_common(targets, m, "targets");
        stk::require(u_out != nullptr, "u_out is NULL");
        stk::require(theta >= 0.0 && theta < 1.0, "theta must be in [0, 1)");
        if (!t->t.have_moments) throw stk::Error(STK_ESTATE, "stk_compute_moments has not been called");
        check_device(t->t.device);
        if (keep_plan) *keep_plan = nullptr;
        auto *pl = new stk_plan();
        try {
            stk::evaluate(t->t, pl->p, targets, m, theta, u_out, false, as_stream(stream));
        } catch (...) {
            delete pl;
            throw;
        }
        if (keep_plan)
            *keep_plan = pl;
        else {
            STK_HIP(hipStreamSynchronize(as_stream(stream)));
            delete pl;
        }
    });
}

stk_status stk_evaluate(const double *targets, int64_t m, const double *sources, int64_t n, const double *f,
                        const double *h, const double *nu, int32_t k_rhs, int32_t p, double theta, int32_t n0,
                        stk_precision prec, double *u_out, stk_plan **keep_plan, void *stream) {
    return guarded([&] {
        check_common(sources, n, "sources");
        check_common(targets, m, "targets");
        stk::require(f && h && nu && u_out, "f, h, nu and u_out must be non-NULL");
        stk::require(n0 >= 1, "n0 must be >= 1");
        stk::require(k_rhs >= 1 && k_rhs <= 64, "k_rhs must be in [1, 64]");
        stk::require(p >= 0 && p <= STK_P_MAX, "p must be in [0, STK_P_MAX]");
        stk::require(prec == STK_FP64 || prec == STK_MIXED, "unknown precision");
        stk::require(theta >= 0.0 && theta < 1.0, "theta must be in [0, 1)");
        if (keep_plan) *keep_plan = nullptr;
        hipStream_t s = as_stream(stream);
        int dev = 0;
        STK_HIP(hipGetDevice(&dev));
        const bool same = targets == sources && m == n;
        if (!keep_plan) {
            // One-shot call: reuse this thread's workspace so that steady-state calls do not
            // allocate.  The workspace lives until the thread ends (never freed: its device
            // memory is returned when the process exits).
            thread_local stk::Tree *ws_tree = nullptr;
            thread_local stk_plan *ws_plan = nullptr;
            if (!ws_tree || ws_tree->device != dev) {
                ws_tree = new stk::Tree();
                ws_plan = new stk_plan();
                ws_tree->device = dev;
            }
            tree_moments_evaluate(*ws_tree, ws_plan->p, targets, m, sources, n, f, h, nu, k_rhs, p, theta, n0, prec,
                                  u_out, same, s);
            STK_HIP(hipStreamSynchronize(s));
            return;
        }
        std::unique_ptr<stk_plan> pl(take_plan(dev));
        if (!pl) {
            pl.reset(new stk_plan());
            pl->p.tree = new stk::Tree();
            pl->p.owns_tree = true;
            pl->p.tree->device = dev;
        }
        tree_moments_evaluate(*pl->p.tree, pl->p, targets, m, sources, n, f, h, nu, k_rhs, p, theta, n0, prec, u_out,
                              same, s);
        *keep_plan = pl.release();
    });
}

stk_status stk_evaluate_regularized(const double *targets, int64_t m, const double *sources, int64_t n,
                                    const double *f, const double *h, const double *nu, double epsilon, int32_t p,
                                    double theta, int32_t n0, double *u_out, void *stream) {
    return guarded([&] {
        check_common(sources, n, "sources");
        check_common(targets, m, "targets");
        stk::require(f && h && nu && u_out, "f, h, nu and u_out must be non-NULL");
        stk::require(n0 >= 1, "n0 must be >= 1");
        stk::require(p >= 0 && p <= STK_P_MAX, "p must be in [0, STK_P_MAX]");
        stk::require(theta >= 0.0 && theta < 1.0, "theta must be in [0, 1)");
        stk::require(std::isfinite(epsilon) && epsilon >= 0.0, "epsilon must be finite and >= 0");
        hipStream_t s = as_stream(stream);
        int dev = 0;
        STK_HIP(hipGetDevice(&dev));
        // this thread's workspace (as the one-shot stk_evaluate): steady-state calls do not
        // allocate; its device memory is returned when the process exits
        thread_local stk::Tree *ws_tree = nullptr;
        thread_local stk_plan *ws_plan = nullptr;
        if (!ws_tree || ws_tree->device != dev) {
            ws_tree = new stk::Tree();
            ws_plan = new stk_plan();
            ws_tree->device = dev;
        }
        stk::build_tree(*ws_tree, sources, n, n0, s);
        stk::compute_moments(*ws_tree, f, h, nu, 1, p, STK_FP64, s);
        stk::evaluate_regularized(*ws_tree, ws_plan->p, targets, m, theta, epsilon, u_out,
                                  targets == sources && m == n, s);
        STK_HIP(hipStreamSynchronize(s));
    });
}

stk_status stk_evaluate_adjoint(stk_plan *plan, const double *w, double *grad_f, double *grad_h,
                                double *grad_targets, double *grad_sources, void *stream) {
    return guarded([&] {
        stk::require(plan != nullptr, "plan is NULL");
        stk::require(w != nullptr, "w is NULL");
        check_device(plan->p.tree->device);
        stk::adjoint(plan->p, w, grad_f, grad_h, grad_targets, grad_sources, as_stream(stream));
    });
}

stk_status stk_direct(const double *targets, int64_t m, const double *sources, int64_t n, const double *f,
                      const double *h, const double *nu, int32_t k_rhs, double *u_out, void *stream) {
    return guarded([&] {
        check_common(targets, m, "targets");
        check_common(sources, n, "sources");
        stk::require(f && h && nu && u_out, "f, h, nu and u_out must be non-NULL");
        stk::require(k_rhs >= 1 && k_rhs <= 64, "k_rhs must be in [1, 64]");
        stk::direct_sum(targets, m, sources, n, f, h, nu, k_rhs, u_out, as_stream(stream));
    });
}

stk_status stk_direct_noalloc(const double *targets, int64_t m, const double *sources, int64_t n, const double *f,
                              const double *h, const double *nu, int32_t k_rhs, double *u_out, void *stream) {
    return guarded([&] {
        check_common(targets, m, "targets");
        check_common(sources, n, "sources");
        stk::require(f && h && nu && u_out, "f, h, nu and u_out must be non-NULL");
        stk::require(k_rhs >= 1 && k_rhs <= 64, "k_rhs must be in [1, 64]");
        stk::direct_sum_noalloc(targets, m, sources, n, f, h, nu, k_rhs, u_out, as_stream(stream));
    });
}

stk_status stk_tree_info(const stk_tree *t, int64_t *nnodes, int32_t *nlevels, double root[4]) {
    return guarded([&] {
        stk::require(t != nullptr, "tree is NULL");
        if (nnodes) *nnodes = t->t.nnodes;
        if (nlevels) *nlevels = t->t.nlevels;
        if (root) {
            for (int a = 0; a < 3; ++a) root[a] = t->t.lo[a];
            root[3] = t->t.L;
        }
    });
}

stk_status stk_tree_export(const stk_tree *t, int32_t *perm, int32_t *level, int32_t *parent, int32_t *child0,
                           int32_t *nchild, int32_t *start, int32_t *count, double *bmin, double *bmax,
                           double *center, double *radius) {
    return guarded([&] {
        stk::require(t != nullptr, "tree is NULL");
        check_device(t->t.device);
        const stk::Tree &T = t->t;
        const size_t nn = size_t(T.nnodes);
        STK_HIP(hipDeviceSynchronize());
        auto cp = [](void *dst, const stk::DBuf &b, size_t bytes) {
            if (dst) STK_HIP(hipMemcpy(dst, b.p, bytes, hipMemcpyDeviceToHost));
        };
        cp(perm, T.perm, sizeof(int32_t) * size_t(T.n));
        cp(level, T.nlevel, sizeof(int32_t) * nn);
        cp(parent, T.nparent, sizeof(int32_t) * nn);
        cp(child0, T.nchild0, sizeof(int32_t) * nn);
        cp(nchild, T.nnchild, sizeof(int32_t) * nn);
        cp(start, T.nstart, sizeof(int32_t) * nn);
        cp(count, T.ncount, sizeof(int32_t) * nn);
        cp(bmin, T.nbmin, sizeof(double) * 3 * nn);
        cp(bmax, T.nbmax, sizeof(double) * 3 * nn);
        cp(center, T.ncenter, sizeof(double) * 3 * nn);
        cp(radius, T.nradius, sizeof(double) * nn);
    });
}

stk_status stk_tree_export_moments(const stk_tree *t, int32_t rhs, double *M, double *Mt) {
    return guarded([&] {
        stk::require(t != nullptr, "tree is NULL");
        const stk::Tree &T = t->t;
        if (!T.have_moments) throw stk::Error(STK_ESTATE, "no moments computed");
        stk::require(rhs >= 0 && rhs < T.k_rhs, "rhs out of range");
        check_device(T.device);
        const int nm = stk::nm_of(T.p);
        const int K = T.k_rhs;
        std::vector<double> h(size_t(T.nnodes) * nm * 12 * K);
        STK_HIP(hipDeviceSynchronize());
        STK_HIP(hipMemcpy(h.data(), T.mom.p, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
        for (size_t c = 0; c < size_t(T.nnodes); ++c)
            for (int a = 0; a < nm; ++a) {
                const double *src = h.data() + (c * nm + a) * 12 * K + 12 * rhs;
                if (M)
                    for (int j = 0; j < 3; ++j) M[(c * nm + a) * 3 + j] = src[j];
                if (Mt)
                    for (int j = 0; j < 9; ++j) Mt[(c * nm + a) * 9 + j] = src[3 + j];
            }
    });
}

stk_status stk_plan_counts(const stk_plan *plan, int64_t *nfar, int64_t *nnear, int64_t *npairs) {
    return guarded([&] {
        stk::require(plan != nullptr, "plan is NULL");
        const stk::Plan &P = plan->p;
        check_device(P.tree->device);
        const size_t m = size_t(P.m);
        std::vector<int32_t> perm(m), a(m), b(m), c(m);
        STK_HIP(hipDeviceSynchronize());
        if (m) STK_HIP(hipMemcpy(perm.data(), P.tperm_p, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
        STK_HIP(hipMemcpy(a.data(), P.cnt_far.p, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
        STK_HIP(hipMemcpy(b.data(), P.cnt_near.p, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
        STK_HIP(hipMemcpy(c.data(), P.cnt_pairs.p, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < m; ++i) {
            if (nfar) nfar[perm[i]] = a[i];
            if (nnear) nnear[perm[i]] = b[i];
            if (npairs) npairs[perm[i]] = c[i];
        }
    });
}

stk_status stk_plan_info(const stk_plan *plan, int64_t *ngroups, int64_t *n_far_entries, int64_t *n_near_entries) {
    return guarded([&] {
        stk::require(plan != nullptr, "plan is NULL");
        if (ngroups) *ngroups = plan->p.ngroups;
        if (n_far_entries) *n_far_entries = plan->p.n_far_entries;
        if (n_near_entries) *n_near_entries = plan->p.n_near_entries;
    });
}

stk_status stk_plan_export_lists(const stk_plan *plan, int32_t kind, int32_t *off, int32_t *node, uint64_t *mask,
                                 int32_t *tperm) {
    return guarded([&] {
        stk::require(plan != nullptr, "plan is NULL");
        stk::require(kind == 0 || kind == 1, "kind must be 0 (far) or 1 (near)");
        const stk::Plan &P = plan->p;
        check_device(P.tree->device);
        STK_HIP(hipDeviceSynchronize());
        const size_t ne = size_t(kind == 0 ? P.n_far_entries : P.n_near_entries);
        auto cp = [](void *dst, const stk::DBuf &b, size_t bytes) {
            if (dst && bytes) STK_HIP(hipMemcpy(dst, b.p, bytes, hipMemcpyDeviceToHost));
        };
        cp(off, kind == 0 ? P.far_off : P.near_off, sizeof(int32_t) * size_t(P.ngroups + 1));
        cp(node, kind == 0 ? P.far_node : P.near_node, sizeof(int32_t) * ne);
        cp(mask, kind == 0 ? P.far_mask : P.near_mask, sizeof(uint64_t) * ne);
        if (tperm && P.m) STK_HIP(hipMemcpy(tperm, P.tperm_p, sizeof(int32_t) * size_t(P.m), hipMemcpyDeviceToHost));
    });
}

}  // extern "C"

namespace {
stk::Tiles from_abi(const stk_tiles &t) {
    stk::Tiles r;
    r.far_kb = t.far_kb;
    r.near_kb = t.near_kb;
    r.near_mfma = t.near_mfma != 0;
    r.far_mfma = t.far_mfma != 0;
    r.far_cm = t.far_cm;
    r.far_split = t.far_split;
    return r;
}
stk_tiles to_abi(const stk::Tiles &t) {
    return stk_tiles{t.far_kb, t.near_kb, t.near_mfma ? 1 : 0, t.far_mfma ? 1 : 0, t.far_cm, t.far_split};
}
void check_tile_key(int32_t p, int32_t k_rhs, stk_precision prec) {
    stk::require(p >= 0 && p <= STK_P_MAX, "p must be in [0, STK_P_MAX]");
    stk::require(k_rhs >= 1 && k_rhs <= 64, "k_rhs must be in [1, 64]");
    stk::require(prec == STK_FP64 || prec == STK_MIXED, "unknown precision");
}
}  // namespace

extern "C" {

stk_status stk_tiles_set(int32_t p, int32_t k_rhs, stk_precision prec, const stk_tiles *tiles) {
    return guarded([&] {
        check_tile_key(p, k_rhs, prec);
        if (!tiles) {
            stk::tiles_set(p, k_rhs, prec, nullptr);
            return;
        }
        const stk::Tiles t = from_abi(*tiles);
        stk::require(stk::tiles_valid(t, k_rhs, prec), "tiles do not fit k_rhs and the precision");
        stk::tiles_set(p, k_rhs, prec, &t);
    });
}

stk_status stk_tiles_get(int32_t p, int32_t k_rhs, stk_precision prec, stk_tiles *out, int32_t *from_table) {
    return guarded([&] {
        check_tile_key(p, k_rhs, prec);
        stk::require(out != nullptr, "out is NULL");
        stk::Tiles t;
        const bool hit = stk::tiles_lookup(p, k_rhs, prec, &t);
        *out = to_abi(hit ? t : stk::default_tiles(k_rhs, prec));
        if (from_table) *from_table = hit ? 1 : 0;
    });
}

stk_status stk_autotune(int32_t p, int32_t k_rhs, stk_precision prec, int64_t n, double theta, int32_t n0,
                        stk_tiles *best, double *best_ms, void *stream) {
    return guarded([&] {
        check_tile_key(p, k_rhs, prec);
        stk::require(n >= 1 && n < (int64_t(1) << 31) / 8, "n out of range");
        stk::require(theta >= 0.0 && theta < 1.0, "theta must be in [0, 1)");
        stk::require(n0 >= 1, "n0 must be >= 1");
        const stk::Tiles t = stk::autotune(p, k_rhs, prec, n, theta, n0, best_ms, as_stream(stream));
        if (best) *best = to_abi(t);
    });
}

stk_status stk_tiles_save(const char *path) {
    return guarded([&] {
        stk::require(path != nullptr, "path is NULL");
        stk::tiles_save(path);
    });
}

stk_status stk_tiles_load(const char *path, int32_t *n_entries) {
    return guarded([&] {
        stk::require(path != nullptr, "path is NULL");
        const int k = stk::tiles_load(path);
        if (n_entries) *n_entries = k;
    });
}

stk_status stk_plan_tiles(const stk_plan *plan, stk_tiles *out) {
    return guarded([&] {
        stk::require(plan != nullptr && out != nullptr, "plan and out must be non-NULL");
        *out = to_abi(plan->p.tiles);
    });
}

stk_status stk_plan_far_split(const stk_plan *plan, int32_t *max_pc, int64_t *sparse_interactions) {
    return guarded([&] {
        stk::require(plan != nullptr, "plan is NULL");
        if (max_pc) *max_pc = plan->p.far_sparse_max;
        if (sparse_interactions) *sparse_interactions = plan->p.far_sparse_max > 0 ? plan->p.fcm.n_inc : 0;
    });
}

stk_status stk_profile_enable(int on) {
    return guarded([&] { stk::prof_enable(on != 0); });
}

stk_status stk_profile_read(double *ms, int64_t *count) {
    return guarded([&] { stk::prof_read(ms, count); });
}

void stk_tree_destroy(stk_tree *t) { delete t; }
void stk_plan_destroy(stk_plan *plan) {
    if (plan) park_or_delete(plan);
}

void stk_plan_cache_clear(void) {
    PlanPool &pp = plan_pool();
    std::vector<stk_plan *> drop;
    {
        std::lock_guard<std::mutex> lk(pp.mu);
        drop.swap(pp.parked);
    }
    for (stk_plan *pl : drop) delete pl;
}

}  // extern "C"
