// tail.hip -- the coarse end of the AMG V-cycle (Sec. 2.2: the
// aggregation-AMG preconditioner) in one workgroup.
//
// Below a few hundred block rows a level's kernels are too small to fill even
// one CU, and every step of the cycle there (restriction, each smoothing
// sweep, the residual, the prolongation, the coarsest solve) costs one kernel
// launch, about 4.5 us on gfx950 even inside a captured graph, most of it
// spent waiting on chains of dependent loads.  From the first such level down
// to the coarsest and back, one workgroup of 1024 threads runs the same steps
// in the same order with workgroup barriers in between.  Everything but the
// matrix values lives in LDS for the whole cycle: the level vectors, the
// sliced-ELL patterns (slice offsets, widths, column indices) and the
// aggregate maps, copied in once at the start.  The values are read from L2
// with several blocks in flight per thread, so a step waits on about one
// memory latency instead of one per block.  The arithmetic of each step is
// that of the multi-kernel path (row sums split over threads and added in the
// same order; only the number of partial sums per row differs), so the two
// agree up to rounding order.
#include "cbs_internal.h"

namespace {

constexpr int kTailThreads = 1024;
// LDS for the staged vectors and index arrays: what a workgroup may hold
// (160 KB on gfx950) less the two static reduction arrays (8 KB in FP32,
// 16 KB in FP64) and 1 KB of margin
constexpr int64_t kTailLdsReserve = 1024;

template <typename T> struct TAcc { using type = double; };
template <> struct TAcc<float> { using type = float; };

// index arrays of a level staged into LDS, in this order
enum { IA_SOFF, IA_SW, IA_SCOL, IA_SOFFO, IA_SWO, IA_SCOLO, IA_APTR, IA_AMEM, IA_AGG, IA_COUNT };
constexpr int kTailCopies = IA_COUNT * kTailMax;

// one level of the tail; offsets are elements into the LDS regions
template <typename T>
struct TailLvl {
    const T *val;                 // values of the full sliced pattern (residual, unscaled sweeps)
    const T *sval;                // values of the row-scaled off-diagonal pattern (scaled sweeps)
    const double *Dinv;           // FP64 inverses of the diagonal blocks
    int32_t ia[IA_COUNT];         // int-region offsets: patterns, restriction lists (rows of
                                  // the finer level per row here), aggregate map (row here ->
                                  // row of the next coarser level)
    int32_t vb, vx, vt, vr, vc;   // vector-region offsets: right side, solution, sweep buffer,
                                  // residual, Dinv b
    int32_t N;                    // block rows
    int32_t lc, lco;              // log2 slice heights of the two patterns
    int32_t sp, spo;              // threads per scalar row on the two patterns
    int32_t scaled;               // sweeps on the row-scaled pattern against c (else with Dinv)
};

template <typename T>
struct TailArgs {
    TailLvl<T> lv[kTailMax];              // smoothed levels, coarsest last (lv[nl])
    const int32_t *csrc[kTailCopies];     // index arrays to stage, in int-region order
    int32_t cpre[kTailCopies + 1];        // their prefix offsets in the int region
    const T *rfine;                       // residual of the level above the tail
    T *xout;                              // where the first tail level's solution goes
    const double *cinv;                   // coarsest: per-system dense inverses
    const int64_t *coff;                  // element offset of each inverse
    const int32_t *cm;                    // order of each system's coarsest matrix
    const int64_t *croff;                 // first scalar row of each system
    double omega;
    int32_t nl, nu1, nu2, nsys;
    int32_t ncopy, nints;                 // staged arrays and their total length
    int32_t ints_off;                     // byte offset of the int region in LDS
};
static_assert(sizeof(TailArgs<double>) <= 4096, "V-cycle tail arguments exceed the kernel-argument limit");

// row r of one block: n contiguous values (16-byte loads for n = 4)
template <int n, typename T>
__device__ inline void tail_load_row(const T *__restrict__ p, T (&v)[n]) {
    if constexpr (n == 4 && sizeof(T) == 4) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 a = *reinterpret_cast<const f4 *>(p);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    } else if constexpr (n == 4 && sizeof(T) == 8) {
        typedef double d2 __attribute__((ext_vector_type(2)));
        const d2 a = *reinterpret_cast<const d2 *>(p), b = *(reinterpret_cast<const d2 *>(p) + 1);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else {
#pragma unroll
        for (int c = 0; c < n; ++c) v[c] = p[c];
    }
}

// copy every index array into the int region, eight elements per thread in
// flight
template <typename T>
__device__ void tail_stage(const TailArgs<T> &a, int32_t *dst) {
    constexpr int U = 8;
    const int t = threadIdx.x;
    for (int32_t g0 = 0; g0 < a.nints; g0 += kTailThreads * U) {
        int32_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t g = g0 + u * kTailThreads + t;
            v[u] = 0;
            if (g < a.nints) {
                int c = 0;
                while (a.cpre[c + 1] <= g) ++c;      // the array holding element g
                v[u] = a.csrc[c][g - a.cpre[c]];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t g = g0 + u * kTailThreads + t;
            if (g < a.nints) dst[g] = v[u];
        }
    }
    __syncthreads();
}

// y = op(from) over all rows of a level; every thread of the workgroup calls
// it.  MODE 1: y = b - A from; 2: y = from + omega Dinv (b - A from);
// 4: y = from + omega (b - from - A from) on the row-scaled values (b = Dinv b).
// sp threads share each scalar row and take its blocks kk, kk + sp, ... (U
// loaded before they are summed, in that order); the partial sums meet in LDS
// and are added in kk order.
template <int n, typename T, int MODE>
__device__ void tail_rows(const int32_t *soff, const int32_t *sw, const int32_t *scol, int lc,
                          const T *__restrict__ val, int sp, int32_t N, const T *from, const T *b, T *y,
                          const double *__restrict__ Dinv, double omega, typename TAcc<T>::type *spart,
                          typename TAcc<T>::type *sres) {
    using A = typename TAcc<T>::type;
    // blocks in flight per thread (more only adds loads of padding: one CU's
    // bandwidth, not the latency, then sets the time)
    constexpr int nn = n * n, U = 4;
    const int tpr = n * sp, R = kTailThreads / tpr;
    const int t = threadIdx.x;
    const int lr = t / tpr, kr = t - lr * tpr;
    const int kk = kr / n, r = kr - kk * n;
    for (int32_t i0 = 0; i0 < N; i0 += R) {
        const int32_t i = i0 + lr;
        const bool act = lr < R && i < N;
        const int32_t o = i * n + r;
        A acc = 0;
        if (act) {
            const int32_t sl = i >> lc, ii = i - (sl << lc);
            const int32_t base = soff[sl] + ii, w = sw[sl];
            for (int32_t k = kk; k < w; k += sp * U) {
                int32_t j[U];
                T bv[U][n];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int32_t kq = k + u * sp;
                    const bool ok = kq < w;
                    const int32_t e = base + ((ok ? kq : kk) << lc);
                    j[u] = ok ? scol[e] : -1;
                    tail_load_row<n, T>(val + (int64_t)e * nn + r * n, bv[u]);
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (j[u] >= 0) {
                        const T *xj = from + j[u] * n;
#pragma unroll
                        for (int c = 0; c < n; ++c) acc += (A)bv[u][c] * (A)xj[c];
                    }
            }
        }
        spart[t] = acc;
        __syncthreads();
        if (act && kk == 0) {
            A sum = 0;
            for (int q = 0; q < sp; ++q) sum += spart[lr * tpr + q * n + r];
            const A res = (A)b[o] - sum;
            if (MODE == 1) {
                y[o] = (T)res;
            } else if (MODE == 4) {
                const A xo = (A)from[o];
                y[o] = (T)(xo + (A)omega * (res - xo));
            } else {
                sres[lr * n + r] = res;
            }
        }
        if (MODE == 2) {
            __syncthreads();
            if (act && kk == 0) {
                const double *Di = Dinv + (int64_t)i * nn + r * n;
                double z = 0.0;
#pragma unroll
                for (int c = 0; c < n; ++c) z += Di[c] * (double)sres[lr * n + c];
                y[o] = (T)((A)from[o] + (A)(omega * z));
            }
        }
        __syncthreads();
    }
}

// b = R rf (rows of the finer level summed in member order); then, when
// sweep0, x = omega Dinv b, and when c is given, c = Dinv b.
template <int n, typename T>
__device__ void tail_restrict(int32_t nc, const int32_t *aptr, const int32_t *amem, const T *rf, T *b,
                              const double *__restrict__ Dinv, double omega, T *x, T *c, bool sweep0,
                              typename TAcc<T>::type *sb) {
    using A = typename TAcc<T>::type;
    constexpr int nn = n * n;
    constexpr int R = kTailThreads / n;
    const int t = threadIdx.x;
    const int lr = t / n, q = t - lr * n;
    const bool dinv = sweep0 || c != nullptr;
    for (int32_t i0 = 0; i0 < nc; i0 += R) {
        const int32_t I = i0 + lr;
        const bool act = lr < R && I < nc;
        const int32_t o = I * n + q;
        A s = 0;
        if (act)
            for (int32_t m = aptr[I]; m < aptr[I + 1]; ++m) s += (A)rf[amem[m] * n + q];
        const T bv = (T)s;
        if (act) b[o] = bv;
        if (dinv) {
            sb[t] = (A)bv;
            __syncthreads();
            if (act) {
                const double *Di = Dinv + (int64_t)I * nn + q * n;
                double z = 0.0;
#pragma unroll
                for (int k = 0; k < n; ++k) z += Di[k] * (double)sb[lr * n + k];
                if (sweep0) x[o] = (T)((A)0 + (A)(omega * z));
                if (c) c[o] = (T)z;
            }
            __syncthreads();
        }
    }
    __syncthreads();
}

template <typename T>
__device__ void tail_fill(int32_t m, T *x) {
    for (int32_t g = threadIdx.x; g < m; g += kTailThreads) x[g] = (T)0;
    __syncthreads();
}

// x += P e: every row takes the correction of its aggregate
template <int n, typename T>
__device__ void tail_prolong(int32_t N, const int32_t *agg, const T *e, T *x) {
    for (int32_t g = threadIdx.x; g < N * n; g += kTailThreads) {
        const int32_t i = g / n;
        const int q = g - i * n;
        x[g] += e[agg[i] * n + q];
    }
    __syncthreads();
}

// coarsest level: x_s = inv_s b_s for every system s, in FP64
template <typename T>
__device__ void tail_coarse(int32_t m_all, const double *__restrict__ inv, const int64_t *__restrict__ off,
                            const int32_t *__restrict__ msz, const int64_t *__restrict__ roff, int32_t nsys,
                            const T *b, T *x) {
    for (int32_t g = threadIdx.x; g < m_all; g += kTailThreads) {
        int32_t lo = 0, hi = nsys - 1;             // last system whose first row is <= g
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (roff[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        const int32_t r0 = (int32_t)roff[lo];
        const int m = msz[lo];
        const double *M = inv + off[lo] + (int64_t)(g - r0) * m;
        double acc = 0.0;
        for (int c = 0; c < m; ++c) acc += M[c] * (double)b[r0 + c];
        x[g] = (T)acc;
    }
    __syncthreads();
}

template <int n, typename T>
__device__ void tail_sweep(const TailLvl<T> &L, const int32_t *is, T *vs, double omega, const T *from, T *to,
                           typename TAcc<T>::type *spart, typename TAcc<T>::type *sres) {
    if (L.scaled)
        tail_rows<n, T, 4>(is + L.ia[IA_SOFFO], is + L.ia[IA_SWO], is + L.ia[IA_SCOLO], L.lco, L.sval, L.spo, L.N,
                           from, vs + L.vc, to, nullptr, omega, spart, sres);
    else
        tail_rows<n, T, 2>(is + L.ia[IA_SOFF], is + L.ia[IA_SW], is + L.ia[IA_SCOL], L.lc, L.val, L.sp, L.N, from,
                           vs + L.vb, to, L.Dinv, omega, spart, sres);
}

// The V-cycle below the level above the tail, same steps as the multi-kernel
// path: per level on the way down a zero-guess sweep fused with the
// restriction, nu1 - 1 more sweeps, the residual; the coarsest solve; per
// level on the way up the prolongation and nu2 sweeps.  Each level's result
// ends in its x (the sweeps alternate between x and t, starting on the one
// that makes the last sweep write x); the first level's x is copied out.
template <int n, typename T>
__global__ __launch_bounds__(kTailThreads) void k_tail(const TailArgs<T> a) {
    using A = typename TAcc<T>::type;
    extern __shared__ __align__(16) char smem[];
    __shared__ A spart[kTailThreads];
    __shared__ A sres[kTailThreads];
    T *vs = reinterpret_cast<T *>(smem);
    int32_t *is = reinterpret_cast<int32_t *>(smem + a.ints_off);
    tail_stage<T>(a, is);
    const int nl = a.nl;
    const int switches = (a.nu1 >= 1 ? a.nu1 - 1 : 0) + a.nu2;
    const int pre_swaps = a.nu1 >= 1 ? a.nu1 - 1 : 0;
    for (int k = 0; k < nl; ++k) {
        const TailLvl<T> &L = a.lv[k];
        T *cur = vs + ((switches % 2 == 0) ? L.vx : L.vt);
        T *oth = vs + ((switches % 2 == 0) ? L.vt : L.vx);
        const T *rf = k == 0 ? a.rfine : vs + a.lv[k - 1].vr;
        const int32_t *aptr = is + L.ia[IA_APTR], *amem = is + L.ia[IA_AMEM];
        T *c = L.scaled ? vs + L.vc : nullptr;
        if (a.nu1 >= 1) {
            tail_restrict<n, T>(L.N, aptr, amem, rf, vs + L.vb, L.Dinv, a.omega, cur, c, true, sres);
            for (int s = 1; s < a.nu1; ++s) {
                tail_sweep<n, T>(L, is, vs, a.omega, cur, oth, spart, sres);
                T *tmp = cur; cur = oth; oth = tmp;
            }
        } else {
            tail_restrict<n, T>(L.N, aptr, amem, rf, vs + L.vb, L.Dinv, a.omega, nullptr, a.nu2 > 0 ? c : nullptr,
                                false, sres);
            tail_fill<T>(L.N * n, cur);
        }
        tail_rows<n, T, 1>(is + L.ia[IA_SOFF], is + L.ia[IA_SW], is + L.ia[IA_SCOL], L.lc, L.val, L.sp, L.N, cur,
                           vs + L.vb, vs + L.vr, nullptr, 0.0, spart, sres);
    }
    {
        const TailLvl<T> &C = a.lv[nl];
        const T *rf = nl == 0 ? a.rfine : vs + a.lv[nl - 1].vr;
        tail_restrict<n, T>(C.N, is + C.ia[IA_APTR], is + C.ia[IA_AMEM], rf, vs + C.vb, nullptr, 0.0, nullptr,
                            nullptr, false, sres);
        tail_coarse<T>(C.N * n, a.cinv, a.coff, a.cm, a.croff, a.nsys, vs + C.vb, vs + C.vx);
    }
    for (int k = nl - 1; k >= 0; --k) {
        const TailLvl<T> &L = a.lv[k];
        T *cur = vs + ((switches % 2 == 0) ? L.vx : L.vt);
        T *oth = vs + ((switches % 2 == 0) ? L.vt : L.vx);
        if (pre_swaps % 2 == 1) { T *tmp = cur; cur = oth; oth = tmp; }
        tail_prolong<n, T>(L.N, is + L.ia[IA_AGG], vs + a.lv[k + 1].vx, cur);
        for (int s = 0; s < a.nu2; ++s) {
            tail_sweep<n, T>(L, is, vs, a.omega, cur, oth, spart, sres);
            T *tmp = cur; cur = oth; oth = tmp;
        }
    }
    const T *x0 = vs + a.lv[0].vx;
    for (int32_t g = threadIdx.x; g < a.lv[0].N * n; g += kTailThreads) a.xout[g] = x0[g];
}

template <typename T> T *vp(DArr<char> &a) { return reinterpret_cast<T *>(a.get()); }

// threads per scalar row in the tail: the largest power of two up to 16 that
// keeps every row of the level in one pass of the workgroup
int32_t tail_split(int32_t N, int n) {
    int32_t sp = 1;
    while (sp < 16 && (int64_t)N * n * sp * 2 <= kTailThreads) sp *= 2;
    return sp;
}

// Lay the tail starting at level l0 out in LDS (vectors of T, then the index
// arrays) and fill the layout part of the arguments; returns the bytes of LDS
// it needs.  With a == nullptr only the size is computed.
template <typename T>
int64_t tail_plan(const cbs_system *h, int l0, bool tr, TailArgs<T> *a) {
    constexpr bool fp32 = sizeof(T) == sizeof(float);
    const int n = h->n;
    const int nlev = (int)h->lev.size();
    const int nl = nlev - 1 - l0;
    auto scaled = [&](const Level &L) { return fp32 && (tr ? L.scaledT : L.scaled); };
    int64_t nvec = 0;                                  // elements of T
    for (int k = 0; k <= nl; ++k) {
        const Level &L = h->lev[l0 + k];
        const bool sc = k < nl && scaled(L);
        const int nv = k == nl ? 2 : (sc ? 5 : 4);
        const int64_t m = (int64_t)L.N * n;
        if (a) {
            TailLvl<T> &d = a->lv[k];
            d.vb = (int32_t)nvec;
            d.vx = (int32_t)(nvec + m);
            if (k < nl) { d.vt = (int32_t)(nvec + 2 * m); d.vr = (int32_t)(nvec + 3 * m); }
            if (sc) d.vc = (int32_t)(nvec + 4 * m);
        }
        nvec += nv * m;
    }
    const int64_t ints_off = (nvec * (int64_t)sizeof(T) + 15) / 16 * 16;
    int64_t nints = 0;
    int ncopy = 0;
    auto add = [&](int k, int which, const int32_t *src, int64_t cnt) {
        if (a) {
            a->lv[k].ia[which] = (int32_t)nints;
            if (cnt > 0) {
                a->csrc[ncopy] = src;
                a->cpre[ncopy] = (int32_t)nints;
                ++ncopy;
            }
        }
        nints += cnt;
    };
    for (int k = 0; k <= nl; ++k) {
        const Level &L = h->lev[l0 + k];
        const Level &F = h->lev[l0 + k - 1];
        if (k < nl) {
            add(k, IA_SOFF, L.sell.soff.get(), (int64_t)L.sell.nslices + 1);
            add(k, IA_SW, L.sell.sw.get(), L.sell.nslices);
            add(k, IA_SCOL, L.sell.scol.get(), L.sell.nent);
            if (scaled(L)) {
                add(k, IA_SOFFO, L.sod.soff.get(), (int64_t)L.sod.nslices + 1);
                add(k, IA_SWO, L.sod.sw.get(), L.sod.nslices);
                add(k, IA_SCOLO, L.sod.scol.get(), L.sod.nent);
            }
            add(k, IA_AGG, L.agg.get(), L.N);
        }
        add(k, IA_APTR, F.agg_ptr.get(), (int64_t)L.N + 1);
        add(k, IA_AMEM, F.agg_mem.get(), F.N);
    }
    if (a) {
        a->cpre[ncopy] = (int32_t)nints;
        a->ncopy = ncopy;
        a->nints = (int32_t)nints;
        a->ints_off = (int32_t)ints_off;
    }
    return ints_off + nints * 4;
}

// dynamic LDS left for the tail: the device's per-workgroup limit (160 KB on
// gfx950) less the kernel's static reduction arrays and a reserve
int64_t tail_budget(const cbs_system *h, size_t tsize) {
    return (int64_t)h->lds_max - 2 * kTailThreads * (int64_t)(tsize == sizeof(float) ? sizeof(float) : sizeof(double)) -
           kTailLdsReserve;
}

}  // namespace

int tail_level_for(const cbs_system *h, size_t tsize) {
    const int nlev = (int)h->lev.size();
    if (nlev < 2 || h->opt.precond != CBS_PREC_AMG) return -1;
    const int32_t lim = h->opt.tail_rows == 0 ? kTailRowsDefault : h->opt.tail_rows;
    if (lim < 0) return -1;
    // a level whose cycle runs twice (W-cycle) keeps its per-step kernels
    for (int l = std::max(1, h->opt.w_levels + 1); l < nlev; ++l) {
        if (h->lev[l].N > lim || nlev - l > kTailMax) continue;
        bool dilu = false;                           // DILU and Gauss-Seidel levels keep their own kernels
        for (int q = l; q + 1 < nlev; ++q) dilu = dilu || h->lev[q].dilu || h->lev[q].sgs;
        if (dilu) continue;
        // the forward layout is the larger one (scaled levels add a pattern and c)
        const int64_t need = tsize == sizeof(float) ? tail_plan<float>(h, l, false, nullptr)
                                                    : tail_plan<double>(h, l, false, nullptr);
        if (need <= tail_budget(h, tsize)) return l;
    }
    return -1;
}

template <typename T>
void launch_tail(cbs_system *h, bool tr, int l0, const T *rfine) {
    constexpr bool fp32 = sizeof(T) == sizeof(float);
    const int n = h->n;
    const int nlev = (int)h->lev.size();
    const int nl = nlev - 1 - l0;
    if (l0 < 1 || nl < 0 || nl + 1 > kTailMax) cbs_throw(CBS_ERR_ARG, "V-cycle tail: bad level range");
    TailArgs<T> a{};
    const int64_t lds = tail_plan<T>(h, l0, tr, &a);
    if (lds > tail_budget(h, sizeof(T))) cbs_throw(CBS_ERR_ARG, "V-cycle tail: LDS budget exceeded");
    for (int k = 0; k <= nl; ++k) {
        Level &L = h->lev[l0 + k];
        TailLvl<T> &d = a.lv[k];
        d.N = L.N;
        if (k == nl) break;                            // the coarsest needs no more
        if constexpr (fp32) d.val = tr ? L.sell.v32T.get() : L.sell.v32.get();
        else d.val = tr ? L.sell.v64T.get() : L.sell.v64.get();
        d.Dinv = tr ? L.DinvT.get() : L.Dinv.get();
        d.lc = L.sell.lc;
        d.sp = tail_split(L.N, n);
        d.scaled = fp32 && (tr ? L.scaledT : L.scaled);
        if (d.scaled) {
            d.sval = reinterpret_cast<const T *>(tr ? L.sod.v32T.get() : L.sod.v32.get());
            d.lco = L.sod.lc;
            d.spo = d.sp;
        }
    }
    Coarse &C = h->coarse;
    a.rfine = rfine;
    a.xout = vp<T>(h->lev[l0].vx);
    a.cinv = tr ? C.invT.get() : C.inv.get();
    a.coff = C.off.get();
    a.cm = C.m.get();
    a.croff = C.roff.get();
    a.omega = level_omega(h->opt, l0);             // every tail level is below level 0
    a.nl = nl;
    a.nu1 = std::max(0, h->opt.pre_sweeps);
    a.nu2 = std::max(0, h->opt.post_sweeps);
    a.nsys = h->n_sys;
    const dim3 g(1), b(kTailThreads);
    const size_t shm = (size_t)lds;
    // more than 64 KB of dynamic LDS is requested explicitly
#define TAIL_N(NN)                                                                                       \
    {                                                                                                    \
        if (shm > 64 * 1024)                                                                             \
            HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_tail<NN, T>),                   \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));           \
        hipLaunchKernelGGL((k_tail<NN, T>), g, b, shm, h->stream, a);                                    \
    }
    switch (n) {
        case 1: TAIL_N(1); break;
        case 2: TAIL_N(2); break;
        case 3: TAIL_N(3); break;
        case 4: TAIL_N(4); break;
        case 5: TAIL_N(5); break;
        default: cbs_throw(CBS_ERR_ARG, "bdim must be 1..5");
    }
#undef TAIL_N
    LAUNCHCHK();
}
template void launch_tail<float>(cbs_system *, bool, int, const float *);
template void launch_tail<double>(cbs_system *, bool, int, const double *);
