// capi.hip -- the extern "C" entry points of libcbs.so (declared in cbs.h).
//
// Lifecycle of Algorithm amgxFoam (Sec. 2.3): create from LDU (pattern +
// values), replace values, set up, solve (warm start), statistics, destroy.
// Every entry point catches internal errors and returns a cbs_status; the
// message goes to a thread-local buffer read by cbs_last_error().
#include "cbs_internal.h"

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <unordered_map>

void globalize_faces(cbs_system *h, const int32_t *la_in, const int32_t *ua_in);
void alloc_krylov(cbs_system *h);

namespace {
thread_local std::string g_last_error;

template <typename F>
int guarded(F &&f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const CbsError &e) {
        g_last_error = e.msg;
        (void)hipGetLastError();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return CBS_ERR_OOM;
    } catch (...) {
        g_last_error = "unexpected internal error";
        return CBS_ERR_HIP;
    }
}

void require(bool cond, int code, const char *msg) {
    if (!cond) cbs_throw(code, msg);
}

double elapsed_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    HIPCHK(hipEventSynchronize(b));
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    return ms;
}

void build_items(cbs_system *h) {
    std::vector<Item> items;
    h->items_per_sys_off.assign(h->n_sys + 1, 0);
    for (int s = 0; s < h->n_sys; ++s) {
        const int64_t b = h->cell_off[s] * h->n, e = h->cell_off[s + 1] * h->n;
        for (int64_t q = b; q < e; q += kItemElems) items.push_back(Item{s, 0, q, std::min<int64_t>(e, q + kItemElems)});
        h->items_per_sys_off[s + 1] = (int32_t)items.size();
    }
    h->n_items = (int32_t)items.size();
    h->items.alloc(items.size());
    HIPCHK(hipMemcpy(h->items.get(), items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice));
    h->item_off.alloc(h->n_sys + 1);
    HIPCHK(hipMemcpy(h->item_off.get(), h->items_per_sys_off.data(), sizeof(int32_t) * (h->n_sys + 1),
                     hipMemcpyHostToDevice));
}


int create_common(cbs_handle *out, int32_t n_sys, const int64_t *cell_off, const int64_t *face_off, int32_t bdim,
                  const int32_t *la, const int32_t *ua, const double *diag, const double *upper, const double *lower,
                  void *stream) {
    require(out != nullptr, CBS_ERR_ARG, "out is NULL");
    *out = nullptr;
    require(bdim >= 1 && bdim <= 5, CBS_ERR_ARG, "bdim must be in 1..5");
    require(n_sys >= 1, CBS_ERR_ARG, "n_sys must be >= 1");
    require(cell_off[0] == 0 && face_off[0] == 0, CBS_ERR_ARG, "offsets must start at 0");
    for (int s = 0; s < n_sys; ++s) {
        require(cell_off[s + 1] > cell_off[s], CBS_ERR_ARG, "every system needs at least one cell");
        require(face_off[s + 1] >= face_off[s], CBS_ERR_ARG, "face offsets must not decrease");
    }
    const int64_t N = cell_off[n_sys], F = face_off[n_sys];
    require(N + 2 * F < (int64_t)INT32_MAX, CBS_ERR_ARG, "too many blocks for 32-bit block indices");
    require(diag != nullptr, CBS_ERR_ARG, "diag is NULL");
    require(F == 0 || (la && ua && upper && lower), CBS_ERR_ARG, "face arrays are NULL");
    set_alloc_stream((hipStream_t)stream);
    std::unique_ptr<cbs_system> h(new cbs_system());
    h->N = (int32_t)N; h->F = (int32_t)F; h->n = bdim; h->n_sys = n_sys;
    h->stream = (hipStream_t)stream;
    HIPCHK(hipGetDevice(&h->device));
    HIPCHK(hipDeviceGetAttribute(&h->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
    h->cell_off.assign(cell_off, cell_off + n_sys + 1);
    h->face_off.assign(face_off, face_off + n_sys + 1);
    HIPCHK(hipEventCreate(&h->ev0));
    HIPCHK(hipEventCreate(&h->ev1));
    h->dflag.alloc(4);
    h->scal.alloc((size_t)S_NSCAL * n_sys);
    h->done.alloc((size_t)3 * n_sys);
    h->flags.alloc((size_t)5 * n_sys);
    HIPCHK(hipMemsetAsync(h->flags.get(), 0, sizeof(int32_t) * 5 * n_sys, h->stream));
    build_items(h.get());
    const auto t0 = std::chrono::steady_clock::now();
    HIPCHK(hipEventRecord(h->ev0, h->stream));
    globalize_faces(h.get(), la, ua);
    convert_pattern(h.get());
    convert_values(h.get(), diag, upper, lower);
    HIPCHK(hipEventRecord(h->ev1, h->stream));
    h->t_convert_ms = elapsed_ms(h->ev0, h->ev1);
    (void)t0;
    *out = h.release();
    return CBS_OK;
}
}  // namespace

[[noreturn]] void cbs_throw(int code, const std::string &msg) { throw CbsError{code, msg}; }

// ------------------------------------------------------------------ memory
// Caching device allocator: a freed block is kept, tagged with the stream
// it was last used on, and handed out again for a request on the same
// stream that fits (up to 2x its size).  Work on one stream runs in order,
// so a block reused on that stream cannot overlap its previous use.  Setup
// re-runs therefore do not free and re-map device memory; cbs_destroy
// returns the handle's cached blocks to HIP.
namespace {
thread_local hipStream_t g_alloc_stream = nullptr;

// the allocator a block came from (all null: hipMalloc / hipFree)
struct AllocHook {
    void *(*alloc)(void *, size_t, void *) = nullptr;
    void (*free)(void *, void *, void *) = nullptr;
    void *ctx = nullptr;
    bool operator==(const AllocHook &o) const { return alloc == o.alloc && free == o.free && ctx == o.ctx; }
};
thread_local AllocHook g_alloc_hook;

struct CachedBlock {
    void *p;
    size_t bytes;
    hipStream_t st;
    AllocHook hook;
};
std::mutex g_mem_mu;
std::multimap<size_t, CachedBlock> g_free_blocks;
std::unordered_map<void *, std::pair<size_t, AllocHook>> g_live_blocks;

void release_block(const CachedBlock &b) {
    if (b.hook.free) b.hook.free(b.hook.ctx, b.p, reinterpret_cast<void *>(b.st));
    else (void)hipFree(b.p);
}
}  // namespace

hipStream_t alloc_stream() { return g_alloc_stream; }
void set_alloc_stream(hipStream_t st) {
    g_alloc_stream = st;
    g_alloc_hook = AllocHook{};
}
// the handle's stream and allocator for the allocations of the current call
static void set_alloc_handle(const cbs_system *h) {
    g_alloc_stream = h->stream;
    g_alloc_hook = AllocHook{h->alloc.alloc, h->alloc.free, h->alloc.ctx};
}

void *dev_alloc(size_t bytes) {
    bytes = (bytes + 511) & ~(size_t)511;
    {
        std::lock_guard<std::mutex> lk(g_mem_mu);
        for (auto it = g_free_blocks.lower_bound(bytes); it != g_free_blocks.end() && it->first <= 2 * bytes; ++it) {
            if (it->second.st != g_alloc_stream || !(it->second.hook == g_alloc_hook)) continue;
            void *p = it->second.p;
            g_live_blocks[p] = {it->first, it->second.hook};
            g_free_blocks.erase(it);
            return p;
        }
    }
    void *q = nullptr;
    if (g_alloc_hook.alloc) {
        q = g_alloc_hook.alloc(g_alloc_hook.ctx, bytes, reinterpret_cast<void *>(g_alloc_stream));
        if (!q) cbs_throw(CBS_ERR_OOM, "the handle's allocator refused " + std::to_string(bytes) + " bytes");
        if (reinterpret_cast<uintptr_t>(q) & 255) {
            g_alloc_hook.free(g_alloc_hook.ctx, q, reinterpret_cast<void *>(g_alloc_stream));
            cbs_throw(CBS_ERR_ARG, "the handle's allocator returned memory not aligned to 256 bytes");
        }
    } else if (hipMalloc(&q, bytes) != hipSuccess || !q) {
        (void)hipGetLastError();
        cbs_throw(CBS_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    std::lock_guard<std::mutex> lk(g_mem_mu);
    g_live_blocks[q] = {bytes, g_alloc_hook};
    return q;
}

void dev_free(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_mem_mu);
    auto it = g_live_blocks.find(p);
    if (it == g_live_blocks.end()) return;
    g_free_blocks.emplace(it->second.first, CachedBlock{p, it->second.first, g_alloc_stream, it->second.second});
    g_live_blocks.erase(it);
}

// return the cached blocks of one stream to the allocators that made them
// (the stream must be idle)
static void dev_cache_trim(hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    for (auto it = g_free_blocks.begin(); it != g_free_blocks.end();) {
        if (it->second.st == st) {
            release_block(it->second);
            it = g_free_blocks.erase(it);
        } else {
            ++it;
        }
    }
}

static double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

PhaseTimer::PhaseTimer(hipStream_t s, const char *w) : st(s), what(w) {
    const char *e = getenv("CBS_PROFILE");
    on = e && e[0] == '1';
    t0 = last = on ? now_ms() : 0.0;
}

void PhaseTimer::mark(const std::string &name) {
    if (!on) return;
    (void)hipStreamSynchronize(st);
    const double t = now_ms();
    marks.emplace_back(name, t - last);
    last = t;
}

PhaseTimer::~PhaseTimer() {
    if (!on) return;
    std::string line = "[cbs] " + what + " total " + std::to_string(last - t0) + " ms:";
    for (auto &m : marks) line += " " + m.first + "=" + std::to_string(m.second).substr(0, 6);
    fprintf(stderr, "%s\n", line.c_str());
}

cbs_system::~cbs_system() {
    if (stream) (void)hipStreamSynchronize(stream);
    else (void)hipDeviceSynchronize();
    invalidate_graphs(this);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
}

extern "C" {

void cbs_default_options(cbs_options *o) {
    if (!o) return;
    o->solver = CBS_SOLVER_BICGSTAB;
    o->restart = 30;
    o->precond = CBS_PREC_AMG;
    o->smoother = CBS_SMOOTH_BJACOBI;
    o->pre_sweeps = 2;
    o->post_sweeps = 2;
    o->omega = 0.9;
    o->tol = 1e-8;
    o->max_iter = 500;
    o->precision = CBS_PRECISION_FP64;
    o->coarse_max = 16;
    o->match_passes = 2;
    o->max_levels = 24;
    o->reuse_aggregates = 0;
    o->check_every = 1;
    o->renumber = 1;
    o->dilu_levels = 2;
    o->row_split = 0;
    o->tail_rows = 0;
    o->schedule = 0;
    o->scaled_sweeps = 1;
    o->w_levels = 0;
    o->coarse_omega = 0.0;
}

int cbs_create_from_ldu(cbs_handle *out, int32_t n_cells, int32_t n_faces, int32_t bdim, const int32_t *lower_addr,
                        const int32_t *upper_addr, const double *diag, const double *upper, const double *lower,
                        void *stream) {
    return guarded([&] {
        require(n_cells >= 1 && n_faces >= 0, CBS_ERR_ARG, "need n_cells >= 1 and n_faces >= 0");
        const int64_t co[2] = {0, n_cells}, fo[2] = {0, n_faces};
        return create_common(out, 1, co, fo, bdim, lower_addr, upper_addr, diag, upper, lower, stream);
    });
}

int cbs_create_batch_from_ldu(cbs_handle *out, int32_t n_sys, const int64_t *cell_off, const int64_t *face_off,
                              int32_t bdim, const int32_t *lower_addr, const int32_t *upper_addr, const double *diag,
                              const double *upper, const double *lower, void *stream) {
    return guarded([&] {
        require(cell_off != nullptr && face_off != nullptr, CBS_ERR_ARG, "offset arrays are NULL");
        return create_common(out, n_sys, cell_off, face_off, bdim, lower_addr, upper_addr, diag, upper, lower, stream);
    });
}

int cbs_update_values(cbs_handle h, const double *diag, const double *upper, const double *lower) {
    return guarded([&] {
        require(h != nullptr, CBS_ERR_ARG, "handle is NULL");
        set_alloc_handle(h);
        require(diag != nullptr && (h->F == 0 || (upper && lower)), CBS_ERR_ARG, "value arrays are NULL");
        HIPCHK(hipEventRecord(h->ev0, h->stream));
        convert_values(h, diag, upper, lower);
        HIPCHK(hipEventRecord(h->ev1, h->stream));
        h->t_convert_ms = elapsed_ms(h->ev0, h->ev1);
        h->values_changed = true;
        h->transposed_ready = false;
        h->valsT.release();
        h->usell.v64.release();
        h->usell.v64T.release();
        invalidate_graphs(h);
        return CBS_OK;
    });
}

int cbs_assemble_luo(cbs_handle h, const double *Q, const double *Sf, const double *lam_visc, const double *v_dt,
                     double gamma) {
    return guarded([&] {
        require(h != nullptr, CBS_ERR_ARG, "handle is NULL");
        set_alloc_handle(h);
        require(h->n == 5, CBS_ERR_ARG, "the density-based assembly needs 5 x 5 blocks");
        require(Q != nullptr && (h->F == 0 || Sf != nullptr), CBS_ERR_ARG, "state or face arrays are NULL");
        require(gamma > 1.0, CBS_ERR_ARG, "gamma must exceed 1");
        HIPCHK(hipEventRecord(h->ev0, h->stream));
        assemble_luo(h, Q, Sf, lam_visc, v_dt, gamma);
        HIPCHK(hipEventRecord(h->ev1, h->stream));
        h->t_convert_ms = elapsed_ms(h->ev0, h->ev1);
        h->values_changed = true;
        h->transposed_ready = false;
        h->valsT.release();
        h->usell.v64.release();
        h->usell.v64T.release();
        invalidate_graphs(h);
        return CBS_OK;
    });
}

int cbs_assemble_luo_noalloc(cbs_handle h, const double *Q, const double *Sf, const double *lam_visc,
                             const double *v_dt, double gamma) {
    return guarded([&] {
        require(h != nullptr, CBS_ERR_ARG, "handle is NULL");
        set_alloc_handle(h);
        require(h->n == 5, CBS_ERR_ARG, "the density-based assembly needs 5 x 5 blocks");
        require(Q != nullptr && (h->F == 0 || Sf != nullptr), CBS_ERR_ARG, "state or face arrays are NULL");
        require(gamma > 1.0, CBS_ERR_ARG, "gamma must exceed 1");
        HIPCHK(hipEventRecord(h->ev0, h->stream));
        assemble_luo_noalloc(h, Q, Sf, lam_visc, v_dt, gamma);
        HIPCHK(hipEventRecord(h->ev1, h->stream));
        h->t_convert_ms = elapsed_ms(h->ev0, h->ev1);
        h->values_changed = true;
        h->transposed_ready = false;
        h->valsT.release();
        h->usell.v64.release();
        h->usell.v64T.release();
        invalidate_graphs(h);
        return CBS_OK;
    });
}

int cbs_assemble_pu(cbs_handle h, const double *Sf, const double *fx, const double *d, const double *flux,
                    const double *nu_eff, const double *vol, const double *uu_add, const double *pp_add) {
    return guarded([&] {
        require(h != nullptr, CBS_ERR_ARG, "handle is NULL");
        set_alloc_handle(h);
        require(h->n == 4, CBS_ERR_ARG, "the pressure-based assembly needs 4 x 4 blocks");
        require(vol != nullptr && (h->F == 0 || (Sf && fx && d && flux && nu_eff)), CBS_ERR_ARG,
                "face or cell arrays are NULL");
        HIPCHK(hipEventRecord(h->ev0, h->stream));
        assemble_pu(h, Sf, fx, d, flux, nu_eff, vol, uu_add, pp_add);
        HIPCHK(hipEventRecord(h->ev1, h->stream));
        h->t_convert_ms = elapsed_ms(h->ev0, h->ev1);
        h->values_changed = true;
        h->transposed_ready = false;
        h->valsT.release();
        h->usell.v64.release();
        h->usell.v64T.release();
        invalidate_graphs(h);
        return CBS_OK;
    });
}

int cbs_setup(cbs_handle h, const cbs_options *opt) {
    return guarded([&] {
        require(h != nullptr, CBS_ERR_ARG, "handle is NULL");
        set_alloc_handle(h);
        cbs_options o;
        if (opt) o = *opt; else cbs_default_options(&o);
        require(o.solver == CBS_SOLVER_BICGSTAB || o.solver == CBS_SOLVER_FGMRES || o.solver == CBS_SOLVER_GMRES,
                CBS_ERR_ARG, "unknown solver");
        require(o.precond >= CBS_PREC_NONE && o.precond <= CBS_PREC_SGS, CBS_ERR_ARG, "unknown preconditioner");
        require(o.smoother >= CBS_SMOOTH_BJACOBI && o.smoother <= CBS_SMOOTH_ILU0, CBS_ERR_ARG, "unknown smoother");
        require(o.precision == CBS_PRECISION_FP64 || o.precision == CBS_PRECISION_MIXED, CBS_ERR_ARG,
                "unknown precision");
        require(o.restart >= 1 && o.restart <= 200, CBS_ERR_ARG, "restart must be in 1..200");
        require(o.tol > 0.0 && o.max_iter >= 0, CBS_ERR_ARG, "need tol > 0 and max_iter >= 0");
        require(o.coarse_max >= 1 && o.max_levels >= 1 && o.match_passes >= 1, CBS_ERR_ARG,
                "coarse_max, max_levels and match_passes must be >= 1");
        require(o.pre_sweeps >= 0 && o.post_sweeps >= 0, CBS_ERR_ARG, "sweeps must be >= 0");
        require(o.row_split == 0 || o.row_split == 1 || o.row_split == 2 || o.row_split == 4 ||
                    o.row_split == 8 || o.row_split == 16,
                CBS_ERR_ARG, "row_split must be 0, 1, 2, 4, 8 or 16");
        require(o.schedule >= 0 && o.schedule <= 6, CBS_ERR_ARG, "schedule must be in 0..6");
        require(o.scaled_sweeps == 0 || o.scaled_sweeps == 1, CBS_ERR_ARG, "scaled_sweeps must be 0 or 1");
        require(o.w_levels >= 0, CBS_ERR_ARG, "w_levels must be >= 0");
        require(o.coarse_omega >= 0.0, CBS_ERR_ARG, "coarse_omega must be >= 0 (0: omega on every level)");
        const bool keep = o.reuse_aggregates && h->setup_done && h->opt.precision == o.precision &&
                          h->opt.precond == o.precond && h->opt.smoother == o.smoother &&
                          h->opt.coarse_max == o.coarse_max && h->opt.match_passes == o.match_passes &&
                          h->opt.max_levels == o.max_levels && h->opt.dilu_levels == o.dilu_levels &&
                          h->opt.renumber == o.renumber && h->opt.scaled_sweeps == o.scaled_sweeps;
        if (!keep) o.reuse_aggregates = 0;
        h->opt = o;
        HIPCHK(hipEventRecord(h->ev0, h->stream));
        h->setup_done = false;
        h->precision_fallback = false;
        invalidate_graphs(h);
        amg_setup(h);
        alloc_krylov(h);
        HIPCHK(hipEventRecord(h->ev1, h->stream));
        h->t_setup_ms = elapsed_ms(h->ev0, h->ev1);
        h->setup_done = true;
        h->values_changed = false;
        return CBS_OK;
    });
}

// Solve; a mixed-precision solve that breaks down or does not converge is
// repeated from the caller's initial guess with the hierarchy in FP64 (same
// aggregates), and the statistics report the escalation.
static int solve_common(cbs_handle h, const double *b, double *x, cbs_stats *st, bool tr) {
    require(h->setup_done && !h->values_changed, CBS_ERR_STATE, "cbs_setup must follow create/update_values");
    const int64_t m = (int64_t)h->N * h->n;
    check_finite(x, m, h->dflag.get(), h->stream);
    const bool mixed = h->opt.precision == CBS_PRECISION_MIXED && h->opt.precond == CBS_PREC_AMG;
    if (mixed) {
        h->x0.ensure(m);
        launch_copy(m, x, h->x0.get(), h->stream);
    }
    int rc = krylov_solve(h, b, x, st, tr);
    if (mixed && rc != CBS_OK) {
        cbs_options o = h->opt;
        o.precision = CBS_PRECISION_FP64;
        o.reuse_aggregates = 1;
        h->opt = o;
        invalidate_graphs(h);
        amg_setup(h);
        alloc_krylov(h);
        h->precision_fallback = true;
        launch_copy(m, h->x0.get(), x, h->stream);
        rc = krylov_solve(h, b, x, st, tr);
    }
    if (st)
        for (int s = 0; s < h->n_sys; ++s) st[s].precision_fallback = h->precision_fallback ? 1 : 0;
    return rc;
}

int cbs_solve(cbs_handle h, const double *b, double *x, cbs_stats *st) {
    return guarded([&] {
        require(h != nullptr && b != nullptr && x != nullptr, CBS_ERR_ARG, "NULL argument");
        set_alloc_handle(h);
        return solve_common(h, b, x, st, false);
    });
}

int cbs_solve_batch(cbs_handle h, const double *b, double *x, cbs_stats *st_array) {
    return guarded([&] {
        require(h != nullptr && b != nullptr && x != nullptr, CBS_ERR_ARG, "NULL argument");
        set_alloc_handle(h);
        return solve_common(h, b, x, st_array, false);
    });
}

int cbs_solve_transpose(cbs_handle h, const double *g, double *lambda, cbs_stats *st) {
    return guarded([&] {
        require(h != nullptr && g != nullptr && lambda != nullptr, CBS_ERR_ARG, "NULL argument");
        set_alloc_handle(h);
        return solve_common(h, g, lambda, st, true);
    });
}

int cbs_gradient(cbs_handle h, const double *lambda, const double *x, double *gd, double *gu, double *gl) {
    return guarded([&] {
        require(h != nullptr && lambda && x && gd && (h->F == 0 || (gu && gl)), CBS_ERR_ARG, "NULL argument");
        set_alloc_handle(h);
        gradient(h, lambda, x, gd, gu, gl);
        HIPCHK(hipStreamSynchronize(h->stream));
        return CBS_OK;
    });
}

int cbs_spmv(cbs_handle h, const double *x, double *y, int32_t transpose) {
    return guarded([&] {
        require(h != nullptr && x && y, CBS_ERR_ARG, "NULL argument");
        set_alloc_handle(h);
        spmv_user(h, x, y, transpose != 0);
        return CBS_OK;
    });
}

int cbs_apply_precond(cbs_handle h, const double *r, double *z) {
    return guarded([&] {
        require(h != nullptr && r && z, CBS_ERR_ARG, "NULL argument");
        set_alloc_handle(h);
        require(h->setup_done && !h->values_changed, CBS_ERR_STATE, "cbs_setup must follow create/update_values");
        if (h->renumbered) {
            const int64_t m = (int64_t)h->N * h->n;
            h->bw.ensure(m);
            h->xw.ensure(m);
            permute_vec(h, r, h->bw.get(), true);
            precond_apply(h, h->bw.get(), h->xw.get(), false);
            permute_vec(h, h->xw.get(), z, false);
        } else {
            precond_apply(h, r, z, false);
        }
        return CBS_OK;
    });
}

int cbs_apply_precond_transpose(cbs_handle h, const double *r, double *z) {
    return guarded([&] {
        require(h != nullptr && r && z, CBS_ERR_ARG, "NULL argument");
        set_alloc_handle(h);
        require(h->setup_done && !h->values_changed, CBS_ERR_STATE, "cbs_setup must follow create/update_values");
        amg_build_transposed(h);
        if (h->renumbered) {
            const int64_t m = (int64_t)h->N * h->n;
            h->bw.ensure(m);
            h->xw.ensure(m);
            permute_vec(h, r, h->bw.get(), true);
            precond_apply(h, h->bw.get(), h->xw.get(), true);
            permute_vec(h, h->xw.get(), z, false);
        } else {
            precond_apply(h, r, z, true);
        }
        return CBS_OK;
    });
}

int cbs_level_apply(cbs_handle h, int32_t level, int32_t op, const void *b, const void *x, void *y, int32_t *fp32) {
    return guarded([&] {
        require(h != nullptr, CBS_ERR_ARG, "handle is NULL");
        set_alloc_handle(h);
        require(h->setup_done && !h->values_changed, CBS_ERR_STATE, "cbs_setup must follow create/update_values");
        require(h->opt.precond == CBS_PREC_AMG, CBS_ERR_STATE, "level kernels need the AMG preconditioner");
        require(level >= 0 && level + 1 < (int32_t)h->lev.size(), CBS_ERR_ARG,
                "level out of range (the coarsest level has no smoother)");
        require(op == CBS_LEVEL_SWEEP || op == CBS_LEVEL_RESIDUAL, CBS_ERR_ARG, "unknown op");
        const bool mixed = h->opt.precision == CBS_PRECISION_MIXED;
        if (fp32) *fp32 = mixed ? 1 : 0;
        if (!b && !x && !y) return CBS_OK;
        require(b && x && y, CBS_ERR_ARG, "NULL vector");
        require(x != y, CBS_ERR_ARG, "y must not alias x");
        Level &L = h->lev[level];
        require(op == CBS_LEVEL_RESIDUAL || (!L.dilu && !L.sgs), CBS_ERR_STATE,
                "a DILU or Gauss-Seidel level has no block-Jacobi sweep");
        const int n = h->n;
        const double w = level_omega(h->opt, level);
        hipStream_t st = h->stream;
        if (mixed) {
            const float *bb = static_cast<const float *>(b), *xx = static_cast<const float *>(x);
            float *yy = static_cast<float *>(y);
            const SellView S = L.sell.view(true);
            if (op == CBS_LEVEL_RESIDUAL)
                launch_rows<float, float>(1, n, S, L.sell.v32.get(), xx, bb, yy, nullptr, 0.0, st);
            else if (L.scaled)
                launch_rows<float, float>(4, n, L.sod.view(true), L.sod.v32.get(), xx, bb, yy, nullptr, w, st);
            else
                launch_rows<float, float>(2, n, S, L.sell.v32.get(), xx, bb, yy, L.Dinv.get(), w, st);
        } else {
            const double *bb = static_cast<const double *>(b), *xx = static_cast<const double *>(x);
            double *yy = static_cast<double *>(y);
            const SellView S = L.sell.view(false);
            if (op == CBS_LEVEL_RESIDUAL)
                launch_rows<double, double>(1, n, S, L.sell.v64.get(), xx, bb, yy, nullptr, 0.0, st);
            else
                launch_rows<double, double>(2, n, S, L.sell.v64.get(), xx, bb, yy, L.Dinv.get(), w, st);
        }
        return CBS_OK;
    });
}

int cbs_pack_fields(int32_t n_cells, int32_t bdim, const double *soa, double *aos, void *stream) {
    return guarded([&] {
        require(n_cells >= 0 && bdim >= 1 && soa && aos, CBS_ERR_ARG, "bad argument");
        pack_fields(n_cells, bdim, soa, aos, (hipStream_t)stream);
        return CBS_OK;
    });
}

int cbs_unpack_fields(int32_t n_cells, int32_t bdim, const double *aos, double *soa, void *stream) {
    return guarded([&] {
        require(n_cells >= 0 && bdim >= 1 && soa && aos, CBS_ERR_ARG, "bad argument");
        unpack_fields(n_cells, bdim, aos, soa, (hipStream_t)stream);
        return CBS_OK;
    });
}

int cbs_get_info(cbs_handle h, int32_t *n_cells, int32_t *n_faces, int32_t *bdim, int64_t *nnzb, int32_t *levels,
                 int32_t *n_sys) {
    return guarded([&] {
        require(h != nullptr, CBS_ERR_ARG, "handle is NULL");
        set_alloc_handle(h);
        if (n_cells) *n_cells = h->N;
        if (n_faces) *n_faces = h->F;
        if (bdim) *bdim = h->n;
        if (nnzb) *nnzb = h->nnzb;
        if (levels) *levels = h->setup_done ? (int32_t)h->lev.size() : 0;
        if (n_sys) *n_sys = h->n_sys;
        return CBS_OK;
    });
}

int cbs_get_bcsr(cbs_handle h, int32_t *row_ptr, int32_t *col, double *vals, int32_t *diag_slot, int32_t *upper_slot,
                 int32_t *lower_slot) {
    return guarded([&] {
        require(h != nullptr, CBS_ERR_ARG, "handle is NULL");
        set_alloc_handle(h);
        hipStream_t st = h->stream;
        const size_t bs = (size_t)h->n * h->n;
        if (row_ptr) HIPCHK(hipMemcpyAsync(row_ptr, h->rp.get(), sizeof(int32_t) * (h->N + 1), hipMemcpyDeviceToDevice, st));
        if (col) HIPCHK(hipMemcpyAsync(col, h->col.get(), sizeof(int32_t) * h->nnzb, hipMemcpyDeviceToDevice, st));
        if (vals) HIPCHK(hipMemcpyAsync(vals, h->vals.get(), sizeof(double) * h->nnzb * bs, hipMemcpyDeviceToDevice, st));
        if (diag_slot) HIPCHK(hipMemcpyAsync(diag_slot, h->dslot.get(), sizeof(int32_t) * h->N, hipMemcpyDeviceToDevice, st));
        if (upper_slot && h->F)
            HIPCHK(hipMemcpyAsync(upper_slot, h->uslot.get(), sizeof(int32_t) * h->F, hipMemcpyDeviceToDevice, st));
        if (lower_slot && h->F)
            HIPCHK(hipMemcpyAsync(lower_slot, h->lslot.get(), sizeof(int32_t) * h->F, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        return CBS_OK;
    });
}

int cbs_get_mirror(cbs_handle h, int32_t *mirror) {
    return guarded([&] {
        require(h != nullptr && mirror != nullptr, CBS_ERR_ARG, "NULL argument");
        set_alloc_handle(h);
        if (h->nnzb > 0)
            HIPCHK(hipMemcpyAsync(mirror, h->mirror.get(), sizeof(int32_t) * h->nnzb, hipMemcpyDeviceToDevice,
                                  h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        return CBS_OK;
    });
}

int cbs_get_level(cbs_handle h, int32_t level, int32_t *n_rows, int64_t *nnzb, int32_t *row_ptr, int32_t *col,
                  double *vals, int32_t *agg, int32_t *colour, int32_t *order) {
    return guarded([&] {
        require(h != nullptr, CBS_ERR_ARG, "handle is NULL");
        set_alloc_handle(h);
        require(h->setup_done, CBS_ERR_STATE, "no hierarchy before cbs_setup");
        require(level >= 0 && level < (int32_t)h->lev.size(), CBS_ERR_ARG, "level out of range");
        Level &L = h->lev[level];
        hipStream_t st = h->stream;
        if (n_rows) *n_rows = L.N;
        if (nnzb) *nnzb = L.nnzb;
        const size_t bs = (size_t)h->n * h->n;
        if (row_ptr) HIPCHK(hipMemcpyAsync(row_ptr, L.rp, sizeof(int32_t) * (L.N + 1), hipMemcpyDeviceToDevice, st));
        if (col) HIPCHK(hipMemcpyAsync(col, L.col, sizeof(int32_t) * L.nnzb, hipMemcpyDeviceToDevice, st));
        if (vals) {
            if (level == 0) level0_values_into(h, vals);
            else HIPCHK(hipMemcpyAsync(vals, L.v64, sizeof(double) * L.nnzb * bs, hipMemcpyDeviceToDevice, st));
        }
        if (agg && L.agg.get()) HIPCHK(hipMemcpyAsync(agg, L.agg.get(), sizeof(int32_t) * L.N, hipMemcpyDeviceToDevice, st));
        if (colour && L.colour.get())
            HIPCHK(hipMemcpyAsync(colour, L.colour.get(), sizeof(int32_t) * L.N, hipMemcpyDeviceToDevice, st));
        if (order) {
            if (L.order.get())
                HIPCHK(hipMemcpyAsync(order, L.order.get(), sizeof(int32_t) * L.N, hipMemcpyDeviceToDevice, st));
            else {
                std::vector<int32_t> id(L.N);
                for (int32_t i = 0; i < L.N; ++i) id[i] = i;
                HIPCHK(hipMemcpyAsync(order, id.data(), sizeof(int32_t) * L.N, hipMemcpyHostToDevice, st));
                HIPCHK(hipStreamSynchronize(st));
            }
        }
        HIPCHK(hipStreamSynchronize(st));
        return CBS_OK;
    });
}

int cbs_set_allocator(cbs_handle h, const cbs_allocator *a) {
    return guarded([&] {
        require(h != nullptr, CBS_ERR_ARG, "handle is NULL");
        require(!a || (a->alloc && a->free), CBS_ERR_ARG, "allocator needs both alloc and free");
        h->alloc = a ? *a : cbs_allocator{};
        return CBS_OK;
    });
}

int cbs_destroy(cbs_handle h) {
    return guarded([&] {
        if (!h) return CBS_OK;
        set_alloc_handle(h);
        hipStream_t st = h->stream;
        delete h;
        dev_cache_trim(st);
        return CBS_OK;
    });
}

const char *cbs_error_string(int code) {
    switch (code) {
        case CBS_OK: return "CBS_OK";
        case CBS_NOT_CONVERGED: return "CBS_NOT_CONVERGED";
        case CBS_ERR_ARG: return "CBS_ERR_ARG";
        case CBS_ERR_PATTERN: return "CBS_ERR_PATTERN";
        case CBS_ERR_SINGULAR: return "CBS_ERR_SINGULAR";
        case CBS_ERR_BREAKDOWN: return "CBS_ERR_BREAKDOWN";
        case CBS_ERR_NONFINITE: return "CBS_ERR_NONFINITE";
        case CBS_ERR_STATE: return "CBS_ERR_STATE";
        case CBS_ERR_OOM: return "CBS_ERR_OOM";
        case CBS_ERR_HIP: return "CBS_ERR_HIP";
        default: return "CBS_UNKNOWN";
    }
}

const char *cbs_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
