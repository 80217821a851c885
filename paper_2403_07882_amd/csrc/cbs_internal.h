// cbs_internal.h -- device runtime shared by the HIP translation units of
// libcbs.so (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <initializer_list>
#include <vector>

#include "cbs.h"

// ---------------------------------------------------------------- errors
struct CbsError {
    int code;
    std::string msg;
};
[[noreturn]] void cbs_throw(int code, const std::string &msg);

#define HIPCHK(x)                                                                    \
    do {                                                                             \
        hipError_t e_ = (x);                                                         \
        if (e_ != hipSuccess)                                                        \
            cbs_throw(CBS_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_));  \
    } while (0)

#define LAUNCHCHK() HIPCHK(hipGetLastError())

// ---------------------------------------------------------------- memory
// Device memory comes from a process-wide cache of hipMalloc blocks: a freed
// block is kept with the stream it was used on (the handle's stream, set by
// set_alloc_stream) and handed out again only to allocations on that stream,
// whose order makes the reuse safe.  Setup can thus allocate and free its
// temporaries without synchronising the device; cbs_destroy returns the
// handle's cached blocks to HIP.
hipStream_t alloc_stream();
void set_alloc_stream(hipStream_t st);
void *dev_alloc(size_t bytes);
void dev_free(void *p);

// Owning device array.  Move-only.
template <typename T>
struct DArr {
    T *p = nullptr;
    size_t n = 0;
    DArr() = default;
    explicit DArr(size_t count) { alloc(count); }
    DArr(const DArr &) = delete;
    DArr &operator=(const DArr &) = delete;
    DArr(DArr &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DArr &operator=(DArr &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DArr() { release(); }
    void alloc(size_t count) {
        release();
        if (count) p = static_cast<T *>(dev_alloc(count * sizeof(T)));
        n = count;
    }
    // allocate only when the current buffer is too small
    void ensure(size_t count) { if (n < count) alloc(count); }
    void release() {
        if (p) dev_free(p);
        p = nullptr; n = 0;
    }
    T *get() const { return p; }
};

// ---------------------------------------------------------------- vectors
// A contiguous range of scalar vector elements belonging to one system.
// Element-wise kernels and reductions run one workgroup per item, so the
// per-system Krylov scalars are loaded once per workgroup.
struct Item {
    int32_t sys;
    int32_t pad;
    int64_t beg, end;
};

constexpr int kItemElems = 4096;      // scalar elements per work item
constexpr int kVecThreads = 256;      // threads per element-wise workgroup

// per-system scalar slots of the Krylov loops: scal[slot * n_sys + s]
enum {
    S_RHO = 0, S_RHO0, S_ALPHA, S_OMEGA, S_RV, S_TS, S_TT, S_RR, S_BB, S_RES0, S_SS,
    S_RRPREV,               // ||r||^2 one iteration earlier (convergence forecast)
    S_RREC,                 // the recurrence's ||r||^2 when the solver stopped (statistics)
    S_NSCAL
};

// ---------------------------------------------------------------- sliced ELL
// Solve-phase storage of a level matrix: slices of C = 2^lc block rows (C =
// kSlice on level 0, kCoarseSlice on coarser levels, where row lengths vary
// more and a shorter slice pads less); in slice s, entry k of row C s + ii
// sits at soff[s] + k C + ii (rows keep
// their column order; short rows are padded with col = -1 up to the slice
// width sw[s]).  One wavefront of a block-row kernel then reads kSlice
// consecutive blocks per step.  BCSR stays the setup-time format.
constexpr int kSlice = 16;
constexpr int kMaxColourRanges = 128;     // colours of a coloured smoother (graph colouring limit)
constexpr int kCoarseSlice = 8;

// Levels with fewer block rows than this are launch- and latency-bound: their
// block-row kernels split rows over several threads, and their first
// post-smoothing sweep absorbs the prolongation.
constexpr int32_t kSmallLevelRows = 65536;
// levels below this many block rows split each scalar row over several
// threads (k_rows_split); larger ones, where one thread per scalar row
// already fills the chip, keep k_rows
constexpr int32_t kSplitLevelRows = 32768;

// block-Jacobi damping of level l: omega on level 0, coarse_omega (when set)
// below it
inline double level_omega(const cbs_options &o, int l) {
    return (l > 0 && o.coarse_omega > 0.0) ? o.coarse_omega : o.omega;
}

// V-cycle tail (tail.hip): default block-row limit of its first level, and the
// most levels (coarsest included) it takes
constexpr int32_t kTailRowsDefault = 256;
constexpr int kTailMax = 8;

// Schedule of the block-row kernels: blocks loaded per step (1, 2, 4) and
// whether matrix values are loaded non-temporally; picked by autotuning.
struct Sched {
    int8_t unroll = 4;
    int8_t nontemporal = 0;
    int8_t split = 1;       // threads sharing one scalar row (1, 2, 4, 8, 16)
};

// Workgroups are dispatched to the eight XCDs in turn (workgroup b to XCD
// b mod 8), each XCD with its own L2.  xcd_block maps the dispatch index to
// a logical one so that each XCD takes one contiguous run of logical
// workgroups (a bijection on 0..G-1): gathers of neighbouring records then
// mostly hit the L2 that already holds them.
__device__ inline uint32_t xcd_block(uint32_t b, uint32_t G) {
    const uint32_t x = b & 7u, k = b >> 3, q = G >> 3, r = G & 7u;
    return x * q + (x < r ? x : r) + k;
}

struct SellView {
    int32_t N;              // row positions (rows, or with prow the padded colour ranges)
    const int32_t *soff, *sw, *scol;
    Sched sched;
    int32_t lc;             // log2 of the slice height
    const int32_t *prow;    // row held at each position (-1: padding); nullptr = identity
};

// Colour-ordered copies (levels with a coloured smoother): position p holds
// row prow[p]; colour c occupies positions cpos[c] .. cpos[c] + (its row
// count), its range padded to whole slices, so one colour's rows are one
// contiguous run of slices.
struct Sell {
    int32_t N = 0, nslices = 0, lc = 4;
    int32_t npos = 0;                     // positions (N when not colour-ordered)
    int64_t nent = 0;
    DArr<int32_t> soff, sw, scol, ssrc;   // ssrc: BCSR slot of each entry, -1 = padding
    DArr<int32_t> prow;                   // colour-ordered: row of each position
    std::vector<int32_t> cpos;            // host, colour-ordered: first position of each colour
    DArr<double> v64, v64T;
    DArr<float> v32, v32T;
    Sched sched64{4, 0}, sched32{4, 1};
    SellView view(bool fp32 = false) const {
        return SellView{npos, soff.get(), sw.get(), scol.get(), fp32 ? sched32 : sched64, lc, prow.get()};
    }
};

// ---------------------------------------------------------------- levels
struct Level {
    int32_t N = 0;          // block rows
    int64_t nnzb = 0;
    // pattern (level 0 points at the handle's arrays)
    int32_t *rp = nullptr, *col = nullptr, *mirror = nullptr, *dslot = nullptr;
    double *v64 = nullptr;  // FP64 values
    float *v32 = nullptr;   // FP32 copy (mixed precision)
    double *v64T = nullptr; // transposed values (adjoint solve)
    float *v32T = nullptr;
    // owned storage (coarse levels own their pattern and values)
    DArr<int32_t> o_rp, o_col, o_mirror, o_dslot;
    DArr<double> o_v64, o_v64T;
    DArr<float> o_v32, o_v32T;
    // per-row system id and per-system row offsets (host copy)
    DArr<int32_t> row_sys;
    std::vector<int64_t> sys_off;
    // smoother data (FP64 per the block-inversion rule)
    DArr<double> Dinv, DinvT;
    // mixed precision, block Jacobi: the FP32 sweeps run on the row-scaled
    // off-diagonal values Dinv_i A_ij, j != i (sod: its own sliced pattern,
    // values in sod.v32), with the level's Dinv b kept in vc
    bool scaled = false;
    Sell sod;
    // the same for the transposed solve: D_i^{-T} (A^T)_ij in sod.v32T, set
    // when the transposed values are built and FP32 holds them all
    bool scaledT = false;
    // DILU: colour classes (rows of colour c: rows_by_colour[colour_off[c] ..
    // colour_off[c+1])) and the FP64 inverses of the DILU diagonal E
    bool dilu = false;
    // symmetric block Gauss-Seidel over the same colour classes (with Dinv)
    bool sgs = false;
    // block ILU(0) (dilu is set too): the unscaled factor F in the BCSR
    // pattern, its sliced copies (FP64, FP32 when mixed) and those of F^T;
    // Einv holds diag(U)^{-1}
    bool ilu = false;
    DArr<double> iluF, iluS64, iluS64T;
    DArr<float> iluS32, iluS32T;
    DArr<int32_t> colour, rows_by_colour;
    std::vector<int32_t> colour_off;     // host, ncolours + 1
    DArr<double> Einv, EinvT;
    // internal renumbering: order[i'] = row of the original numbering
    DArr<int32_t> order;
    // level 0 without its own values in the internal numbering (a
    // block-Jacobi level 0): its sliced copies and block inverses read the
    // caller's block CSR (h->vals) through slot maps composed with the
    // renumbering (the patterns' ssrc, and dslot_src for the diagonal
    // blocks); v64 is then null, or after a values-only re-setup the
    // internal copy the Galerkin product of level 1 reads
    bool lazy_vals = false;
    DArr<int32_t> dslot_src;
    // transfer to the next level
    DArr<int32_t> agg, agg_ptr, agg_mem;
    int32_t nc = 0;
    int32_t maxc = 0;                    // largest Galerkin candidate list of the aggregation
    // level vectors in the hierarchy precision (bytes)
    DArr<char> vb, vx, vr, vt, vc;
    // solve-phase matrix copy
    Sell sell;
};

struct Coarse {
    DArr<double> inv;                    // per-system dense inverses, concatenated
    DArr<double> invT;
    DArr<int64_t> off;                   // element offset of each system's inverse
    DArr<int32_t> m;                     // order of each system's matrix (rows * n)
    DArr<int64_t> roff;                  // scalar-row offset of each system
    int32_t max_m = 0;
};

// ---------------------------------------------------------------- handle
struct cbs_system {
    int32_t N = 0, F = 0, n = 0, n_sys = 1;
    int device = 0;                              // device current at creation (holds every buffer)
    int lds_max = 64 * 1024;                     // LDS bytes one workgroup may hold on that device
    cbs_allocator alloc{};                       // the caller's allocator (all null: hipMalloc)
    hipStream_t stream = nullptr;
    std::vector<int64_t> cell_off, face_off;     // host
    // level-0 pattern and conversion maps
    DArr<int32_t> la, ua;                        // face addresses, global cell ids
    DArr<int32_t> rp, col, src, mirror, dslot, uslot, lslot;
    DArr<double> vals;                           // FP64 block CSR values
    // device assembly scratch: per-face and per-cell passes (density-based:
    // S lambda; u, v, w, H, phi; net face vector and sum of S lambda;
    // pressure-based: Rhie-Chow and diffusion coefficients; pp diagonal;
    // a_uu, D and the up/pu diagonal vector)
    DArr<double> face_lam, cell_prim, cell_acc;
    int64_t nnzb = 0;
    // preconditioner
    bool setup_done = false, values_changed = false, transposed_ready = false;
    cbs_options opt{};
    std::vector<Level> lev;
    Coarse coarse;
    double op_complexity = 1.0;
    // Krylov workspace (FP64, N*n each)
    DArr<double> r, rh, p, v, ph, s, sh, t, w;
    DArr<double> V, Z, H, gvec, cs, sn, yv;      // FGMRES
    DArr<double> scal, partial;                  // per-system scalars, reduction partials
    DArr<int32_t> done, flags;                   // per-system converged / breakdown flags
    DArr<Item> items;                            // element ranges for level-0 vectors
    int32_t n_items = 0;
    std::vector<int32_t> items_per_sys_off;      // host: first item of each system
    DArr<int32_t> item_off;                      // device copy of the above
    DArr<int32_t> dflag;                         // error flag scratch for checks
    // pinned host mirrors for read-back
    double *h_scal = nullptr;
    int32_t *h_done = nullptr;
    // captured iteration graphs (index: transposed solve), replayed on `stream`
    hipStream_t cap_stream = nullptr;
    // captured BiCGStab iteration: [whole, first half, second half][forward, transposed]
    hipGraphExec_t g_iter[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
    DArr<double> xw, bw;                         // solution / rhs work copies the graphs point at
    // internal renumbering of level 0 (AMG setup)
    bool renumbered = false;
    DArr<int32_t> perm_sk;                       // permuted level-0 slot -> caller-order slot
    DArr<double> valsT;                          // caller-order A^T values (cbs_spmv transpose)
    Sell usell;                                  // caller-order sliced copy (cbs_spmv)
    // mixed precision escalated to FP64 (sticky until the next cbs_setup)
    bool precision_fallback = false;
    DArr<double> x0;                             // caller's initial guess, kept for a re-solve
    // statistics
    double t_convert_ms = 0.0, t_setup_ms = 0.0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    ~cbs_system();
};

// ---------------------------------------------------------------- helpers
inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// Phase timers for setup and solve, printed to stderr when the environment
// sets CBS_PROFILE=1 (each mark synchronises the stream, so only then).
struct PhaseTimer {
    bool on;
    hipStream_t st;
    double t0, last;
    std::vector<std::pair<std::string, double>> marks;
    PhaseTimer(hipStream_t s, const char *what);
    void mark(const std::string &name);
    ~PhaseTimer();
    std::string what;
};

// exclusive scan of n int32 counts into out[0..n] (out[n] = total); in may alias out
void scan_exclusive(const int32_t *in, int32_t *out, int64_t n, hipStream_t st);
int32_t read_int(const int32_t *dptr, hipStream_t st);
// several device int32 scalars / a short device array, one synchronisation
constexpr int kPinnedWords = 64;
int32_t *pinned_words();                 // kPinnedWords pinned host words of this thread
void read_ints(std::initializer_list<const int32_t *> src, int32_t *out, hipStream_t st);
void read_array(const int32_t *dptr, int32_t count, int32_t *out, hipStream_t st);

// conversion (convert.hip)
void convert_pattern(cbs_system *h);
void convert_values(cbs_system *h, const double *diag, const double *upper, const double *lower);
void assemble_luo(cbs_system *h, const double *Q, const double *Sf, const double *lam_visc, const double *v_dt,
                  double gamma);
// allocation-free variant of assemble_luo on the library's fixed scratch
// (kNoAllocScratchBytes per device; larger systems are refused)
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
size_t assemble_luo_scratch_bytes(int64_t N, int64_t F);
void assemble_luo_noalloc(cbs_system *h, const double *Q, const double *Sf, const double *lam_visc,
                          const double *v_dt, double gamma);
void assemble_pu(cbs_system *h, const double *Sf, const double *fx, const double *d, const double *flux,
                 const double *nu, const double *vol, const double *uu_add, const double *pp_add);
void check_finite(const double *a, int64_t count, int32_t *dflag, hipStream_t st);
void pack_fields(int32_t N, int32_t n, const double *soa, double *aos, hipStream_t st);
void unpack_fields(int32_t N, int32_t n, const double *aos, double *soa, hipStream_t st);
void gradient(cbs_system *h, const double *lam, const double *x, double *gd, double *gu, double *gl);

// block-row kernels (spmv.hip).  T = FP64 or FP32 level precision.
//   mode 0: y = A x;  mode 1: y = b - A x;  mode 2: y = x + omega Dinv (b - A x)
//   mode 3: y = omega Dinv b (block-Jacobi sweep from a zero guess), and
//           aux = Dinv b when aux is not null
//   mode 4: y = x + omega (b - x - A x) on the row-scaled off-diagonal values
//           Dinv_i A_ij (j != i) with b = Dinv b: the sweep of mode 2
// Modes 2 and 4 with pagg != nullptr sweep from x + P e (pagg: aggregate map
// of the level, pe: coarse-level correction): the prolongation fused into
// the first post-smoothing sweep.
// Modes 2 and 4 with y64 != nullptr write the result widened to FP64 into y64
// instead of y.
template <typename TV, typename TX>
void launch_rows(int mode, int n, const SellView &S, const TV *val, const TX *x, const TX *b, TX *y,
                 const double *Dinv, double omega, hipStream_t st, TX *aux = nullptr,
                 const int32_t *pagg = nullptr, const TX *pe = nullptr, double *y64 = nullptr);
// Mixed precision, level 0: b = FP32(b64) fused with the zero-guess sweep
// x = omega Dinv b (and c = Dinv b when c is not null).
void launch_cast_sweep0(int n, int32_t N, const double *b64, float *b, const double *Dinv, double omega, float *x,
                        float *c, hipStream_t st);
// Restriction fused into the zero-guess block-Jacobi sweep of the coarse
// level: b[I] = sum of r over the members of aggregate I (agg_ptr/agg_mem of
// the fine level, summed in member order like launch_restrict), then
// x = omega Dinv b and, when c is not null, c = Dinv b.
template <typename TX>
void launch_restrict_sweep0(int n, int32_t nc, const int32_t *agg_ptr, const int32_t *agg_mem, const TX *r, TX *b,
                            const double *Dinv, double omega, TX *x, TX *c, hipStream_t st);
// time the schedules of the residual kernel on S (cached per shape)
Sched autotune_rows(int n, const Sell &S, bool fp32, const void *val, hipStream_t st);
// the schedule option: 0 = autotune_rows, 1..6 = a forced (unroll, non-temporal) pair
Sched choose_sched(int n, const Sell &S, bool fp32, const void *val, int32_t forced, hipStream_t st);
// threads per scalar row of the block-row kernels on a level (row_split option)
int8_t row_split_for(const Sell &S, int64_t nblocks, int32_t opt_split);
// sliced-ELL pattern from BCSR (offdiag: without the diagonal blocks), and
// values gathered from BCSR values
void sell_build(int32_t N, const int32_t *rp, const int32_t *col, Sell &S, hipStream_t st, bool offdiag = false,
                int slice = kSlice, const int32_t *rows_by_colour = nullptr,
                const std::vector<int32_t> *colour_off = nullptr);
// the same in two halves, so that several patterns share one read-back of
// their entry counts (S.soff[S.nslices] after begin)
// slice: slice height, a power of two up to 64
// rows_by_colour / colour_off (host): build the copy colour-ordered
void sell_pattern_begin(int32_t N, const int32_t *rp, const int32_t *col, Sell &S, hipStream_t st, bool offdiag,
                        int slice = kSlice, const int32_t *rows_by_colour = nullptr,
                        const std::vector<int32_t> *colour_off = nullptr);
void sell_pattern_finish(const int32_t *rp, const int32_t *col, Sell &S, int64_t nent, hipStream_t st,
                         bool offdiag);
// (with out32: also the FP32 rounding of every value, bit 64 of *flag set for
// values FP32 cannot hold)
void sell_fill(int n, const Sell &S, const double *bcsr_vals, double *out, hipStream_t st, float *out32 = nullptr,
               int32_t *flag = nullptr);
// out = FP32(Dinv_i A_ij) for every entry of the sliced pattern S, A_ij read
// from the block-CSR values; an entry FP32 cannot hold sets bit 64 of *flag
void sell_scale(int n, const Sell &S, const double *bcsr_vals, const double *Dinv, float *out, int32_t *flag,
                hipStream_t st);
// sell_fill (FP64 + FP32) of the full pattern F and sell_scale of the
// off-diagonal pattern O of the same level in one pass over the values
// (F and O built with the same slice height, not colour-ordered)
void sell_fill_scaled(int n, const Sell &F, const Sell &O, const double *bcsr_vals, const double *Dinv,
                      double *f64, float *f32, float *o32, int32_t *flag, hipStream_t st);
template <typename TX>
void launch_restrict(int n, int32_t nc, const int32_t *agg_ptr, const int32_t *agg_mem,
                     const TX *r, TX *bc, hipStream_t st);
template <typename TX>
void launch_prolong(int n, int32_t N, const int32_t *agg, const TX *e, TX *x, hipStream_t st);
template <typename TA, typename TB>
void launch_cast(int64_t m, const TA *a, TB *b, hipStream_t st);
void launch_coarse_solve(cbs_system *h, bool transposed, const void *b, void *x, bool fp32);
void launch_block_apply(int n, int32_t N, const double *Dinv, const double *r, double *z, hipStream_t st);
// V-cycle tail (tail.hip): the first level (>= 1) from which the rest of the
// cycle runs in one workgroup for level vectors of tsize bytes per value, or
// -1; and that launch, given the residual of the level above (the result
// lands in the first tail level's x)
int tail_level_for(const cbs_system *h, size_t tsize);
template <typename T>
void launch_tail(cbs_system *h, bool tr, int l0, const T *rfine);
// block Gauss-Seidel on the cnt rows of one colour, held at positions
// p0 .. p0 + cnt of the colour-ordered copy S, in place, with the pivot
// inverses Dinv (D or E): form 0 x_i = P_i^{-1} (b_i - sum_{j != i} A_ij x_j),
// form 1 x_i += P_i^{-1} (b_i - sum_j A_ij x_j), form 2 x_i = P_i^{-1} b_i
// (no matrix read); rz (optional) gets zeros at the rows written
template <typename T>
void launch_gs_colour(int n, const SellView &S, const T *val, int32_t p0, int32_t cnt, const double *Dinv,
                      const T *b, T *x, hipStream_t st, int form = 0, T *rz = nullptr);
// DILU colour sweeps on the cnt rows at positions p0 .. p0 + cnt: forward
// y = E^{-1}(b - A x - L y) (zero_guess: A x omitted; last: also x = x + y,
// the last colour's whole update), backward z = y - E^{-1} U z, x = x + z
template <typename T>
void launch_dilu_fwd(int n, const SellView &S, const T *val, const T *fval, const int32_t *colour, int c, int32_t p0,
                     int32_t cnt, const double *Einv, const T *b, T *x, T *y, bool zero_guess, bool last,
                     hipStream_t st);
template <typename T>
void launch_dilu_bwd(int n, const SellView &S, const T *val, const int32_t *colour, int c, int32_t p0, int32_t cnt,
                     const double *Einv, T *yz, T *x, bool zero_guess, hipStream_t st);

// AMG setup (amg.hip)
void amg_setup(cbs_system *h);
void amg_build_transposed(cbs_system *h);
// lazy0: keep no internal copy of the level-0 values (see Level::lazy_vals)
void renumber_hierarchy(cbs_system *h, int32_t *deferred, bool lazy0);
// level-0 values in the internal numbering into out[nnzb * n * n]
void level0_values_into(cbs_system *h, double *out);
void refresh_level0_values(cbs_system *h);
void permute_vec(cbs_system *h, const double *in, double *out, bool to_internal);
void spmv_user(cbs_system *h, const double *x, double *y, bool transposed);
// block-diagonal inverses of level l; with bad_slot the first singular block
// row is left there for the caller to check, else it is checked here
// (dslot: slots of the diagonal blocks in vals, default the level's own)
void blockinv_level(cbs_system *h, int l, const double *vals, double *Dinv, int32_t *bad_slot = nullptr,
                    const int32_t *dslot = nullptr);

// Krylov (krylov.hip)
int krylov_solve(cbs_system *h, const double *b, double *x, cbs_stats *st, bool transposed);
void invalidate_graphs(cbs_system *h);
void launch_copy(int64_t m, const double *a, double *b, hipStream_t st);
template <typename T>
void launch_fill(int64_t m, T *a, hipStream_t st);
void precond_apply(cbs_system *h, const double *r, double *z, bool transposed);
void spmv64(cbs_system *h, const double *x, double *y, bool transposed);
