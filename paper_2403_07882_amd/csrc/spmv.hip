// spmv.hip -- block-row kernels: block SpMV, residual, block-Jacobi sweeps,
// restriction / prolongation, precision casts and the coarsest-level solve.
//
// Block SpMV of the coupled system (Eq. coupl_system): y_i = sum_j A_ij x_j
// over block CSR with dense n x n row-major blocks (Sec. 2.3).  Mapping for
// gfx950: one workgroup = 64 block rows x n threads; thread (row i, r) owns
// scalar row i*n + r and streams the r-th row of each block of block row i
// (n contiguous values).  The n threads of a block row read the whole block
// (n*n contiguous values) together, so every fetched cache line is used in
// full; x_j is gathered once per block and shared through L1.  Smoother
// modes finish with D_i^{-1} (FP64) applied to the n residual components of
// the block row, exchanged through LDS.
#include "cbs_internal.h"

#include <map>
#include <mutex>
#include <tuple>

namespace {

template <typename T> struct Acc { using type = double; };
template <> struct Acc<float> { using type = float; };

typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// Row r of one block: n contiguous values, streamed once per SpMV, so they
// are loaded non-temporally (keeps x resident in the caches).  16-byte
// vector loads where the alignment allows it (n = 4).
// Row r of one block (n contiguous values), loaded non-temporally when NT
// (values are streamed once per sweep); 16-byte vector loads for n = 4.
template <int n, typename T, bool NT>
__device__ inline void load_row_nt(const T *__restrict__ p, T (&v)[n]) {
    if constexpr (n == 4 && sizeof(T) == 8) {
        const dbl2 a = NT ? __builtin_nontemporal_load(reinterpret_cast<const dbl2 *>(p))
                          : *reinterpret_cast<const dbl2 *>(p);
        const dbl2 b = NT ? __builtin_nontemporal_load(reinterpret_cast<const dbl2 *>(p) + 1)
                          : *(reinterpret_cast<const dbl2 *>(p) + 1);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else if constexpr (n == 4 && sizeof(T) == 4) {
        const flt4 a = NT ? __builtin_nontemporal_load(reinterpret_cast<const flt4 *>(p))
                          : *reinterpret_cast<const flt4 *>(p);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    } else {
#pragma unroll
        for (int c = 0; c < n; ++c) v[c] = NT ? __builtin_nontemporal_load(p + c) : p[c];
    }
}

// default schedule of the DILU sweeps: streamed FP32, cached FP64
template <int n, typename T>
__device__ inline void load_block_row(const T *__restrict__ p, T (&v)[n]) {
    load_row_nt<n, T, sizeof(T) == 4>(p, v);
}

template <int n, typename T>
__device__ inline void load_x(const T *__restrict__ p, T (&v)[n]) {
#pragma unroll
    for (int c = 0; c < n; ++c) v[c] = p[c];
}
template <>
__device__ inline void load_x<4, double>(const double *__restrict__ p, double (&v)[4]) {
    const dbl2 a = *reinterpret_cast<const dbl2 *>(p), b = *(reinterpret_cast<const dbl2 *>(p) + 1);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
template <>
__device__ inline void load_x<4, float>(const float *__restrict__ p, float (&v)[4]) {
    const flt4 a = *reinterpret_cast<const flt4 *>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

// x_j as a sweep sees it: with PRO the coarse-grid correction of j's
// aggregate, e[agg[j]], is added first -- the same floating-point addition the
// prolongation kernel makes, so fusing prolongation into the first
// post-smoothing sweep changes no result.
template <int n, typename TX, bool PRO>
__device__ inline void load_xc(const TX *__restrict__ x, int64_t j, const int32_t *__restrict__ pagg,
                               const TX *__restrict__ pe, TX (&v)[n]) {
    load_x<n, TX>(x + j * n, v);
    if constexpr (PRO) {
        const TX *ej = pe + (int64_t)pagg[j] * n;
#pragma unroll
        for (int c = 0; c < n; ++c) v[c] = v[c] + ej[c];
    }
}

// mode 0: y = A x; 1: y = b - A x; 2: y = x + w Dinv (b - A x); 3: y = w Dinv b
// (and aux = Dinv b when aux is given); 4: y = x + w (b - x - A x), the sweep
// of mode 2 on the row-scaled off-diagonal values Dinv_i A_ij (j != i; the
// scaled diagonal block is the identity and is not stored) with b = Dinv b.
// Rows are read from the sliced-ELL copy: at step k the C rows of a slice
// (C = 16 on level 0, 8 on coarser levels) read C consecutive blocks; U steps
// are loaded before they are summed, and the sums run in the row's column
// order.
// Modes 2 and 4 with PRO: x is first corrected by the prolongated coarse
// solution (x + P e, pagg = aggregate map, pe = e), see load_xc.
template <int n, typename TV, typename TX, int MODE, int U, bool NT, bool PRO>
__global__ __launch_bounds__(64 * n) void k_rows(SellView S, const TV *__restrict__ val, const TX *__restrict__ x,
                                                 const TX *__restrict__ b, TX *__restrict__ y,
                                                 const double *__restrict__ Dinv, double omega,
                                                 TX *__restrict__ aux, const int32_t *__restrict__ pagg,
                                                 const TX *__restrict__ pe, double *__restrict__ y64) {
    using A = typename Acc<TX>::type;
    constexpr int nn = n * n;
    const int t = threadIdx.x;
    const int lr = t / n, r = t - lr * n;
    // position p in the sliced copy holds block row i (colour-ordered copies
    // map positions to rows; the padding positions of their colour ranges
    // hold none)
    const int32_t p = blockIdx.x * 64 + lr;
    const int32_t i = (S.prow && p < S.N) ? S.prow[p] : p;
    const bool act = p < S.N && i >= 0;
    // sweep result: to y, or widened to FP64 into y64 (the last sweep of a
    // mixed-precision V-cycle hands its result straight to the FP64 loop)
    auto put = [&](int64_t o, TX v) {
        if (y64) y64[o] = (double)v;
        else y[o] = v;
    };
    A acc = 0;
    if (MODE != 3 && act) {
        const int32_t sl = p >> S.lc, ii = p - (sl << S.lc);
        const int32_t base = S.soff[sl] + ii, w = S.sw[sl];
        int32_t k = 0;
        for (; k + U <= w; k += U) {
            int32_t j[U];
            TV bv[U][n];
            TX xv[U][n];
#pragma unroll
            for (int u = 0; u < U; ++u) j[u] = S.scol[base + ((k + u) << S.lc)];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t e = base + ((int64_t)(k + u) << S.lc);
                load_row_nt<n, TV, NT>(val + e * nn + r * n, bv[u]);
                load_xc<n, TX, PRO>(x, j[u] < 0 ? i : j[u], pagg, pe, xv[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (j[u] >= 0) {
#pragma unroll
                    for (int c = 0; c < n; ++c) acc += (A)bv[u][c] * (A)xv[u][c];
                }
        }
        for (; k < w; ++k) {
            const int64_t e = base + ((int64_t)k << S.lc);
            const int32_t j = S.scol[e];
            if (j < 0) continue;
            TV bv[n];
            TX xv[n];
            load_row_nt<n, TV, NT>(val + e * nn + r * n, bv);
            load_xc<n, TX, PRO>(x, j, pagg, pe, xv);
#pragma unroll
            for (int c = 0; c < n; ++c) acc += (A)bv[c] * (A)xv[c];
        }
    }
    const int64_t o = (int64_t)i * n + r;
    auto x_own = [&]() -> A {
        TX v = x[o];
        if constexpr (PRO) v = v + pe[(int64_t)pagg[i] * n + r];
        return (A)v;
    };
    if (MODE == 0) {
        if (act) y[o] = (TX)acc;
        return;
    }
    A res = 0;
    if (act) res = (A)b[o] - acc;
    if (MODE == 1) {
        if (act) y[o] = (TX)res;
        return;
    }
    if (MODE == 4) {
        if (act) {
            const A xo = x_own();
            put(o, (TX)(xo + (A)omega * (res - xo)));
        }
        return;
    }
    __shared__ A sres[64 * n];
    sres[t] = res;
    __syncthreads();
    if (act) {
        const double *Di = Dinv + (int64_t)i * nn + r * n;
        double z = 0.0;
#pragma unroll
        for (int c = 0; c < n; ++c) z += Di[c] * (double)sres[lr * n + c];
        const A xi = (MODE == 2) ? x_own() : (A)0;
        put(o, (TX)(xi + (A)(omega * z)));
        if (MODE == 3 && aux) aux[o] = (TX)z;
    }
}

// Coarse levels have few block rows with many blocks each, so the chain of
// dependent loads (column, then x) along a row, not bandwidth, sets the time.
// Here SP threads share each scalar row: thread kk takes blocks kk, kk + SP,
// ...; the SP partial sums meet in LDS and are added in kk order.  A
// workgroup covers 64 / SP block rows.
template <int n, typename TV, typename TX, int MODE, int SP, bool PRO>
__global__ __launch_bounds__(64 * n) void k_rows_split(SellView S, const TV *__restrict__ val,
                                                       const TX *__restrict__ x, const TX *__restrict__ b,
                                                       TX *__restrict__ y, const double *__restrict__ Dinv,
                                                       double omega, [[maybe_unused]] TX *__restrict__ aux,
                                                       const int32_t *__restrict__ pagg,
                                                       const TX *__restrict__ pe, double *__restrict__ y64) {
    using A = typename Acc<TX>::type;
    constexpr int nn = n * n, R = 64 / SP;
    auto put = [&](int64_t o, TX v) {
        if (y64) y64[o] = (double)v;
        else y[o] = v;
    };
    const int t = threadIdx.x;
    const int lr = t / (n * SP), kr = t - lr * (n * SP);
    const int kk = kr / n, r = kr - kk * n;
    const int32_t p = blockIdx.x * R + lr;
    const int32_t i = (S.prow && p < S.N) ? S.prow[p] : p;
    const bool act = p < S.N && i >= 0;
    A acc = 0;
    if (act) {
        const int32_t sl = p >> S.lc, ii = p - (sl << S.lc);
        const int32_t base = S.soff[sl] + ii, w = S.sw[sl];
        for (int32_t k = kk; k < w; k += SP) {
            const int64_t e = base + ((int64_t)k << S.lc);
            const int32_t j = S.scol[e];
            if (j < 0) continue;
            TV bv[n];
            TX xv[n];
            load_row_nt<n, TV, false>(val + e * nn + r * n, bv);
            load_xc<n, TX, PRO>(x, j, pagg, pe, xv);
#pragma unroll
            for (int c = 0; c < n; ++c) acc += (A)bv[c] * (A)xv[c];
        }
    }
    auto x_own = [&](int64_t o) -> A {
        TX v = x[o];
        if constexpr (PRO) v = v + pe[(int64_t)pagg[i] * n + r];
        return (A)v;
    };
    __shared__ A spart[64 * n];
    __shared__ A sres[R * n];
    spart[t] = acc;
    __syncthreads();
    const int64_t o = (int64_t)i * n + r;
    if (kk == 0) {
        A sum = 0;
#pragma unroll
        for (int q = 0; q < SP; ++q) sum += spart[lr * n * SP + q * n + r];
        if (MODE == 0) {
            if (act) y[o] = (TX)sum;
        } else {
            const A res = act ? (A)b[o] - sum : (A)0;
            if (MODE == 1) {
                if (act) y[o] = (TX)res;
            } else if (MODE == 4) {
                if (act) {
                    const A xo = x_own(o);
                    put(o, (TX)(xo + (A)omega * (res - xo)));
                }
            } else {
                sres[lr * n + r] = res;
            }
        }
    }
    if (MODE != 2) return;
    __syncthreads();
    if (kk == 0 && act) {
        const double *Di = Dinv + (int64_t)i * nn + r * n;
        double z = 0.0;
#pragma unroll
        for (int c = 0; c < n; ++c) z += Di[c] * (double)sres[lr * n + c];
        put(o, (TX)(x_own(o) + (A)(omega * z)));
    }
}

template <int n, typename TV, typename TX, int MODE, bool PRO>
void rows_launch(const SellView &S, const TV *val, const TX *x, const TX *b, TX *y, const double *Dinv,
                 double omega, TX *aux, const int32_t *pagg, const TX *pe, double *y64, hipStream_t st) {
    const dim3 g(cdiv(S.N, 64)), bl(64 * n);
    const int u = S.sched.unroll;
    const bool nt = S.sched.nontemporal != 0;
#define ROWS_V(UU, NTT)                                                                                  \
    hipLaunchKernelGGL((k_rows<n, TV, TX, MODE, UU, NTT, PRO>), g, bl, 0, st, S, val, x, b, y, Dinv, omega, \
                       aux, pagg, pe, y64)
    if (MODE == 3) { ROWS_V(1, false); return; }       // no matrix read
    const int sp = S.sched.split;
    if (sp > 1) {
        const dim3 gs(cdiv((int64_t)S.N * sp, 64));
#define ROWS_S(SS)                                                                                           \
    hipLaunchKernelGGL((k_rows_split<n, TV, TX, MODE, SS, PRO>), gs, bl, 0, st, S, val, x, b, y, Dinv, omega, \
                       aux, pagg, pe, y64)
        if (sp == 2) ROWS_S(2);
        else if (sp == 4) ROWS_S(4);
        else if (sp == 8) ROWS_S(8);
        else ROWS_S(16);
#undef ROWS_S
        return;
    }
    if (u <= 1) { if (nt) ROWS_V(1, true); else ROWS_V(1, false); }
    else if (u == 2) { if (nt) ROWS_V(2, true); else ROWS_V(2, false); }
    else { if (nt) ROWS_V(4, true); else ROWS_V(4, false); }
#undef ROWS_V
}

template <int n, typename TV, typename TX, int MODE>
void rows_nm(const SellView &S, const TV *val, const TX *x, const TX *b, TX *y, const double *Dinv, double omega,
             TX *aux, const int32_t *pagg, const TX *pe, double *y64, hipStream_t st) {
    if constexpr (MODE == 2 || MODE == 4) {
        if (pagg) {
            rows_launch<n, TV, TX, MODE, true>(S, val, x, b, y, Dinv, omega, aux, pagg, pe, y64, st);
            return;
        }
    }
    rows_launch<n, TV, TX, MODE, false>(S, val, x, b, y, Dinv, omega, aux, nullptr, nullptr, y64, st);
}

template <int n, typename TV, typename TX>
void rows_n(int mode, const SellView &S, const TV *val, const TX *x, const TX *b, TX *y, const double *Dinv,
            double omega, TX *aux, const int32_t *pagg, const TX *pe, double *y64, hipStream_t st) {
    switch (mode) {
        case 0: rows_nm<n, TV, TX, 0>(S, val, x, b, y, Dinv, omega, aux, pagg, pe, y64, st); break;
        case 1: rows_nm<n, TV, TX, 1>(S, val, x, b, y, Dinv, omega, aux, pagg, pe, y64, st); break;
        case 2: rows_nm<n, TV, TX, 2>(S, val, x, b, y, Dinv, omega, aux, pagg, pe, y64, st); break;
        case 3: rows_nm<n, TV, TX, 3>(S, val, x, b, y, Dinv, omega, aux, pagg, pe, y64, st); break;
        case 4: rows_nm<n, TV, TX, 4>(S, val, x, b, y, Dinv, omega, aux, pagg, pe, y64, st); break;
    }
}

// ------------------------------------------------------------------ DILU sweeps
constexpr int kDiluU = 4;    // blocks in flight per thread in the coloured sweeps

// Multicolour DILU (one launch per colour): rows of colour c depend only on
// rows of other colours, which earlier launches finished.
//   forward  y_i = E_i^{-1} (b_i - sum_j A_ij x_j - sum_{colour(j) < c} A_ij y_j)
//   backward z_i = y_i - E_i^{-1} sum_{colour(j) > c} A_ij z_j ;  x_i += z_i
// so x + z = x + M^{-1}(b - A x) with M = (E + L) E^{-1} (E + U).  One
// thread per (row, r) as in k_rows; E^{-1} (FP64) is applied through LDS.
// One colour of a block Gauss-Seidel half-sweep, in place: for the rows of
// colour c (rows[0..cnt)), x_i = P_i^{-1} (b_i - sum_{j != i} A_ij x_j), with
// the pivot P = D (Gauss-Seidel) or E (DILU).  Rows of one colour are not
// neighbours, so each reads only x of other colours and writes only its own.
// FORM 1 is the correction x_i += P_i^{-1} (b_i - sum_j A_ij x_j), the
// diagonal included; FORM 2 is x_i = P_i^{-1} b_i, for when every neighbour
// is still zero (no matrix read).  rz, when given, gets zeros at the rows
// written: their residual, known to vanish.
template <int n, typename T, int FORM>
__global__ __launch_bounds__(64 * n) void k_gs_colour(SellView S, const T *__restrict__ val, int32_t p0,
                                                      int32_t cnt, const double *__restrict__ Dinv,
                                                      const T *__restrict__ b, T *x, T *__restrict__ rz) {
    using A = typename Acc<T>::type;
    constexpr int nn = n * n;
    const int t = threadIdx.x;
    const int lr = t / n, r = t - lr * n;
    const int32_t q = blockIdx.x * 64 + lr;
    const bool act = q < cnt;
    const int32_t p = p0 + q;                     // the colour's rows are one run of positions
    const int32_t i = act ? S.prow[p] : 0;
    A acc = 0;
    if (act && FORM != 2) {
        const int32_t sl = p >> S.lc, ii = p - (sl << S.lc);
        const int32_t base = S.soff[sl] + ii, w = S.sw[sl];
        // kDiluU blocks in flight per step, summed in column order;
        // padding (column -1) adds nothing, nor the diagonal outside FORM 1
        for (int32_t k0 = 0; k0 < w; k0 += kDiluU) {
            int32_t j[kDiluU];
            T bv[kDiluU][n], xv[kDiluU][n];
#pragma unroll
            for (int u = 0; u < kDiluU; ++u)
                j[u] = k0 + u < w ? S.scol[base + ((int64_t)(k0 + u) << S.lc)] : -1;
#pragma unroll
            for (int u = 0; u < kDiluU; ++u) {
                if (j[u] < 0 || (FORM == 0 && j[u] == i)) continue;
                load_block_row<n, T>(val + (base + ((int64_t)(k0 + u) << S.lc)) * nn + r * n, bv[u]);
                load_x<n, T>(x + (int64_t)j[u] * n, xv[u]);
            }
#pragma unroll
            for (int u = 0; u < kDiluU; ++u) {
                if (j[u] < 0 || (FORM == 0 && j[u] == i)) continue;
#pragma unroll
                for (int cc = 0; cc < n; ++cc) acc += (A)bv[u][cc] * (A)xv[u][cc];
            }
        }
    }
    __shared__ A sres[64 * n];
    sres[t] = act ? (A)b[(int64_t)i * n + r] - acc : (A)0;
    __syncthreads();
    if (act) {
        const double *Di = Dinv + (int64_t)i * nn + r * n;
        double z = 0.0;
#pragma unroll
        for (int cc = 0; cc < n; ++cc) z += Di[cc] * (double)sres[lr * n + cc];
        const int64_t o = (int64_t)i * n + r;
        if (FORM == 1) x[o] = (T)((A)x[o] + (A)(T)z);
        else x[o] = (T)z;
        if (rz) rz[o] = (T)0;
    }
}

// fval: the lower-triangle values when they differ from val (block ILU(0):
// val = A for the residual, fval = its factor), else nullptr
// LAST (the last colour, which has no upper neighbours): the backward step
// leaves its y unchanged, so x_i += y_i is made here and the backward launch
// of that colour is skipped.  Rows of one colour are not neighbours, so
// writing x_i here cannot change what another row of the colour reads.
template <int n, typename T, bool ZERO, bool LAST>
__global__ __launch_bounds__(64 * n) void k_dilu_fwd(SellView S, const T *__restrict__ val,
                                                     const T *__restrict__ fval,
                                                     const int32_t *__restrict__ colour, int c, int32_t p0,
                                                     int32_t cnt, const double *__restrict__ Einv,
                                                     const T *__restrict__ b, T *x, T *__restrict__ y) {
    using A = typename Acc<T>::type;
    constexpr int nn = n * n;
    const int t = threadIdx.x;
    const int lr = t / n, r = t - lr * n;
    const int32_t q = blockIdx.x * 64 + lr;
    const bool act = q < cnt;
    const int32_t p = p0 + q;                     // the colour's rows are one run of positions
    const int32_t i = act ? S.prow[p] : 0;
    A ax = 0, ay = 0;
    if (act) {
        const int32_t sl = p >> S.lc, ii = p - (sl << S.lc);
        const int32_t base = S.soff[sl] + ii, w = S.sw[sl];
        // kDiluU blocks in flight per step, summed in column order
        for (int32_t k0 = 0; k0 < w; k0 += kDiluU) {
            int32_t j[kDiluU];
            bool lo[kDiluU];
            T bv[kDiluU][n], xv[kDiluU][n], yv[kDiluU][n], fv[kDiluU][n];
#pragma unroll
            for (int u = 0; u < kDiluU; ++u)
                j[u] = k0 + u < w ? S.scol[base + ((int64_t)(k0 + u) << S.lc)] : -1;
#pragma unroll
            for (int u = 0; u < kDiluU; ++u) {
                // two colours (colour == nullptr): every neighbour of a
                // colour-1 row precedes it
                lo[u] = j[u] >= 0 && (colour ? colour[j[u]] < c : (c == 1 && j[u] != i));
                if (j[u] < 0) continue;
                const int64_t e = base + ((int64_t)(k0 + u) << S.lc);
                load_block_row<n, T>(val + e * nn + r * n, bv[u]);
                if (!ZERO) load_x<n, T>(x + (int64_t)j[u] * n, xv[u]);
                if (lo[u]) {
                    load_x<n, T>(y + (int64_t)j[u] * n, yv[u]);
                    if (fval) load_block_row<n, T>(fval + e * nn + r * n, fv[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < kDiluU; ++u) {
                if (j[u] < 0) continue;
                if (!ZERO) {
#pragma unroll
                    for (int cc = 0; cc < n; ++cc) ax += (A)bv[u][cc] * (A)xv[u][cc];
                }
                if (lo[u]) {
#pragma unroll
                    for (int cc = 0; cc < n; ++cc) ay += (A)(fval ? fv[u][cc] : bv[u][cc]) * (A)yv[u][cc];
                }
            }
        }
    }
    __shared__ A sres[64 * n];
    sres[t] = act ? (A)b[(int64_t)i * n + r] - ax - ay : (A)0;
    __syncthreads();
    if (act) {
        const double *Ei = Einv + (int64_t)i * nn + r * n;
        double z = 0.0;
#pragma unroll
        for (int cc = 0; cc < n; ++cc) z += Ei[cc] * (double)sres[lr * n + cc];
        const int64_t o = (int64_t)i * n + r;
        y[o] = (T)z;
        if (LAST) x[o] = ZERO ? (T)z : (T)((A)x[o] + (A)(T)z);
    }
}

template <int n, typename T, bool ZERO>
__global__ __launch_bounds__(64 * n) void k_dilu_bwd(SellView S, const T *__restrict__ val,
                                                     const int32_t *__restrict__ colour, int c, int32_t p0,
                                                     int32_t cnt, const double *__restrict__ Einv,
                                                     T *__restrict__ yz, T *__restrict__ x) {
    using A = typename Acc<T>::type;
    constexpr int nn = n * n;
    const int t = threadIdx.x;
    const int lr = t / n, r = t - lr * n;
    const int32_t q = blockIdx.x * 64 + lr;
    const bool act = q < cnt;
    const int32_t p = p0 + q;
    const int32_t i = act ? S.prow[p] : 0;
    A au = 0;
    if (act) {
        const int32_t sl = p >> S.lc, ii = p - (sl << S.lc);
        const int32_t base = S.soff[sl] + ii, w = S.sw[sl];
        // kDiluU blocks in flight per step, summed in column order; only
        // neighbours of later colours count
        for (int32_t k0 = 0; k0 < w; k0 += kDiluU) {
            int32_t j[kDiluU];
            bool up[kDiluU];
            T bv[kDiluU][n], zv[kDiluU][n];
#pragma unroll
            for (int u = 0; u < kDiluU; ++u)
                j[u] = k0 + u < w ? S.scol[base + ((int64_t)(k0 + u) << S.lc)] : -1;
#pragma unroll
            for (int u = 0; u < kDiluU; ++u) {
                up[u] = j[u] >= 0 && (colour ? colour[j[u]] > c : (c == 0 && j[u] != i));
                if (!up[u]) continue;
                load_block_row<n, T>(val + (base + ((int64_t)(k0 + u) << S.lc)) * nn + r * n, bv[u]);
                load_x<n, T>(yz + (int64_t)j[u] * n, zv[u]);
            }
#pragma unroll
            for (int u = 0; u < kDiluU; ++u) {
                if (!up[u]) continue;
#pragma unroll
                for (int cc = 0; cc < n; ++cc) au += (A)bv[u][cc] * (A)zv[u][cc];
            }
        }
    }
    __shared__ A su[64 * n];
    su[t] = au;
    __syncthreads();
    if (act) {
        const double *Ei = Einv + (int64_t)i * nn + r * n;
        double d = 0.0;
#pragma unroll
        for (int cc = 0; cc < n; ++cc) d += Ei[cc] * (double)su[lr * n + cc];
        const int64_t o = (int64_t)i * n + r;
        const A z = (A)yz[o] - (A)d;
        yz[o] = (T)z;
        x[o] = ZERO ? (T)z : (T)((A)x[o] + z);
    }
}

// ------------------------------------------------------------------ sliced ELL build
// offdiag: leave out the diagonal block of each row (counted, not assumed)
// Slice widths: one thread per (padded) row computes its stored length, the
// C consecutive lanes of a slice (C divides the wavefront) take the maximum.
__global__ void k_sell_width(int32_t npos, int32_t ns, int32_t C, const int32_t *rp, const int32_t *col,
                             const int32_t *prow, int32_t *sw, int32_t *cnt, int offdiag) {
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t i = p < npos ? (prow ? prow[p] : p) : -1;
    int32_t len = 0;
    if (i >= 0) {
        len = rp[i + 1] - rp[i];
        if (offdiag)
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k) len -= col[k] == i ? 1 : 0;
    }
    for (int o = C >> 1; o > 0; o >>= 1) len = max(len, __shfl_xor(len, o, 64));
    const int32_t sl = p / C;
    if (p - sl * C == 0 && sl < ns) {
        sw[sl] = len;
        cnt[sl] = len * C;
    }
}

__global__ void k_sell_fill_idx(int32_t npos, int32_t C, const int32_t *rp, const int32_t *col, const int32_t *prow,
                                const int32_t *soff, int32_t *scol, int32_t *ssrc, int offdiag) {
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npos) return;
    const int32_t i = prow ? prow[p] : p;
    if (i < 0) return;
    const int32_t sl = p / C, ii = p - sl * C;
    int32_t q = 0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        if (offdiag && col[k] == i) continue;
        const int64_t e = soff[sl] + (int64_t)q * C + ii;
        scol[e] = col[k];
        ssrc[e] = k;
        ++q;
    }
}

__global__ void k_fill_i32(int64_t m, int32_t *a, int32_t v) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < m) a[g] = v;
}

// Colour-ordered positions: the t-th row of the (colour, row)-sorted list
// goes to position cpos[c] + t - off[c] of its colour c.
struct ColourRanges {
    int32_t ncol;
    int32_t off[kMaxColourRanges + 1], cpos[kMaxColourRanges + 1];
};

__global__ void k_colour_positions(int32_t N, ColourRanges cr, const int32_t *rows, int32_t *prow) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    int lo = 0, hi = cr.ncol - 1;            // colour c with off[c] <= t < off[c+1]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cr.off[mid] <= t) lo = mid; else hi = mid - 1;
    }
    prow[cr.cpos[lo] + (t - cr.off[lo])] = rows[t];
}

// Values of a sliced copy gathered from block CSR (zeros in padding); with
// out32, also their FP32 rounding, flagging (bit 64) values FP32 cannot hold.
// Each thread moves kSellV(n) consecutive values of one block: 4 or 2 when
// n*n allows, else one block row (odd n).
__host__ __device__ constexpr int kSellV(int n) { return (n * n) % 4 == 0 ? 4 : ((n * n) % 2 == 0 ? 2 : n); }

template <int n, bool F32>
__global__ void k_sell_vals(int64_t nent, const int32_t *__restrict__ ssrc, const double *__restrict__ in,
                            double *__restrict__ out, float *__restrict__ out32, int32_t *flag) {
    constexpr int nn = n * n, V = kSellV(n);
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nent * (nn / V)) return;
    const int64_t e = g / (nn / V);
    const int64_t o = e * nn + (g - e * (nn / V)) * V;     // first value of this thread
    const int32_t k = ssrc[e];
    const double *src = in + (int64_t)(k < 0 ? 0 : k) * nn + (o - e * nn);
    double v[V];
#pragma unroll
    for (int c = 0; c < V; ++c) v[c] = k >= 0 ? src[c] : 0.0;
    bool bad = false;
#pragma unroll
    for (int c = 0; c < V; ++c) {
        out[o + c] = v[c];
        if constexpr (F32) {
            const float f = (float)v[c];
            out32[o + c] = f;
            bad = bad || !isfinite(f);
        }
    }
    if (bad) atomicOr(flag, 64);
}

// Row-scaled FP32 values for the block-Jacobi sweep: entry (i, j) of the
// sliced copy S becomes Dinv_i A_ij (A_ij read from the block-CSR values
// through S.ssrc), formed in FP64 and rounded once.  One thread per (slice
// row, r); padding entries, including the rows that pad the last slice past
// N, get zeros.
constexpr int kScaleU = 4;   // entries per row staged together in k_sell_scaled

template <int n>
__global__ __launch_bounds__(64 * n) void k_sell_scaled(int32_t N, int32_t nslices, int32_t lc,
                                                        const int32_t *__restrict__ soff,
                                                        const int32_t *__restrict__ sw,
                                                        const int32_t *__restrict__ ssrc,
                                                        const double *__restrict__ bvals,
                                                        const double *__restrict__ Dinv, float *__restrict__ out,
                                                        int32_t *flag) {
    // 64 slice rows per workgroup, n threads each; per entry, thread r stages
    // row r of the block A_ij in LDS and then forms row r of Dinv_i A_ij from
    // all of it (each block is read from memory once).  kScaleU entries of a
    // row are staged at a time, so their loads are in flight together.
    constexpr int nn = n * n;
    constexpr int U = kScaleU;
    __shared__ double sa[U * 64 * nn];
    __shared__ int32_t wmax;
    const int t = threadIdx.x, lr = t / n, r = t - lr * n;
    const int64_t npos = (int64_t)nslices << lc;
    const int64_t i = (int64_t)blockIdx.x * 64 + lr;
    const bool act = i < npos;
    const int32_t sl = act ? (int32_t)(i >> lc) : 0;
    const int64_t base = act ? (int64_t)soff[sl] + (i - ((int64_t)sl << lc)) : 0;
    const int32_t w = act ? sw[sl] : 0;
    if (t == 0) wmax = 0;
    __syncthreads();
    if (r == 0 && w > 0) atomicMax(&wmax, w);
    double d[n];
#pragma unroll
    for (int q = 0; q < n; ++q) d[q] = (act && i < N) ? Dinv[i * nn + r * n + q] : 0.0;
    __syncthreads();
    const int32_t W = wmax;
    bool bad = false;
    for (int32_t k0 = 0; k0 < W; k0 += U) {
        int32_t src[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = base + ((int64_t)(k0 + u) << lc);
            src[u] = (k0 + u < w && i < N) ? ssrc[e] : -1;
        }
        double a[U][n];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double *p = bvals + (int64_t)(src[u] < 0 ? 0 : src[u]) * nn + r * n;
#pragma unroll
            for (int c = 0; c < n; ++c) a[u][c] = src[u] < 0 ? 0.0 : p[c];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int c = 0; c < n; ++c) sa[(u * 64 + lr) * nn + r * n + c] = a[u][c];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (k0 + u >= w) continue;
            const int64_t e = base + ((int64_t)(k0 + u) << lc);
#pragma unroll
            for (int c = 0; c < n; ++c) {
                double acc = 0.0;
#pragma unroll
                for (int q = 0; q < n; ++q) acc += d[q] * sa[(u * 64 + lr) * nn + q * n + c];
                const float v = (float)acc;
                out[e * nn + r * n + c] = v;
                bad = bad || !isfinite(v);
            }
        }
        __syncthreads();
    }
    if (bad) atomicOr(flag, 64);
}

// Both sliced copies of a mixed block-Jacobi level in one pass over its
// FP64 block-CSR values: the full pattern F (FP64 values and their FP32
// rounding, as k_sell_vals) and the off-diagonal pattern O (FP32 of
// Dinv_i A_ij, as k_sell_scaled).  F and O share their slices (the same
// rows at the same positions); every row holds its diagonal block, so
// O's slot of a block is F's slot less one once the diagonal has passed,
// and F's padding slots past a row's end cover O's.  One thread per (slice
// row, r), kScaleU entries staged in LDS at a time.
template <int n>
__global__ __launch_bounds__(64 * n) void k_sell_fill_scaled(int32_t N, int32_t nslices, int32_t lc,
                                                             const int32_t *__restrict__ fsoff,
                                                             const int32_t *__restrict__ fsw,
                                                             const int32_t *__restrict__ fscol,
                                                             const int32_t *__restrict__ fssrc,
                                                             const int32_t *__restrict__ osoff,
                                                             const int32_t *__restrict__ osw,
                                                             const double *__restrict__ bvals,
                                                             const double *__restrict__ Dinv,
                                                             double *__restrict__ f64, float *__restrict__ f32,
                                                             float *__restrict__ o32, int32_t *flag) {
    constexpr int nn = n * n;
    constexpr int U = kScaleU;
    __shared__ double sa[U * 64 * nn];
    __shared__ int32_t wmax;
    const int t = threadIdx.x, lr = t / n, r = t - lr * n;
    const int64_t npos = (int64_t)nslices << lc;
    const int64_t i = (int64_t)blockIdx.x * 64 + lr;
    const bool act = i < npos;
    const int32_t sl = act ? (int32_t)(i >> lc) : 0;
    const int64_t ii = act ? i - ((int64_t)sl << lc) : 0;
    const int64_t fbase = act ? (int64_t)fsoff[sl] + ii : 0, obase = act ? (int64_t)osoff[sl] + ii : 0;
    const int32_t w = act ? fsw[sl] : 0, wo = act ? osw[sl] : 0;
    if (t == 0) wmax = 0;
    __syncthreads();
    if (r == 0 && w > 0) atomicMax(&wmax, w);
    double d[n];
#pragma unroll
    for (int q = 0; q < n; ++q) d[q] = (act && i < N) ? Dinv[i * nn + r * n + q] : 0.0;
    __syncthreads();
    const int32_t W = wmax;
    bool bad = false;
    int32_t passed = 0;                                // 1 once this row's diagonal block has gone by
    for (int32_t k0 = 0; k0 < W; k0 += U) {
        int32_t src[U], cj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = fbase + ((int64_t)(k0 + u) << lc);
            const bool in = k0 + u < w && i < N;
            src[u] = in ? fssrc[e] : -1;
            cj[u] = in ? fscol[e] : -1;
        }
        double a[U][n];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double *p = bvals + (int64_t)(src[u] < 0 ? 0 : src[u]) * nn + r * n;
#pragma unroll
            for (int c = 0; c < n; ++c) a[u][c] = src[u] < 0 ? 0.0 : p[c];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int c = 0; c < n; ++c) sa[(u * 64 + lr) * nn + r * n + c] = a[u][c];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (k0 + u >= w) continue;
            const int64_t e = fbase + ((int64_t)(k0 + u) << lc);
#pragma unroll
            for (int c = 0; c < n; ++c) {
                f64[e * nn + r * n + c] = a[u][c];
                const float v = (float)a[u][c];
                f32[e * nn + r * n + c] = v;
                bad = bad || !isfinite(v);
            }
            const bool diag = cj[u] == (int32_t)i;
            if (diag) { passed = 1; continue; }
            const int32_t jo = k0 + u - passed;
            if (jo >= wo) continue;
            const int64_t eo = obase + ((int64_t)jo << lc);
#pragma unroll
            for (int c = 0; c < n; ++c) {
                double acc = 0.0;
#pragma unroll
                for (int q = 0; q < n; ++q) acc += d[q] * sa[(u * 64 + lr) * nn + q * n + c];
                const float v = (float)acc;
                o32[eo * nn + r * n + c] = v;
                bad = bad || !isfinite(v);
            }
        }
        __syncthreads();
    }
    if (bad) atomicOr(flag, 64);
}

template <typename TX>
__global__ void k_restrict(int32_t nc, int n, const int32_t *__restrict__ aptr, const int32_t *__restrict__ amem,
                           const TX *__restrict__ r, TX *__restrict__ bc) {
    using A = typename Acc<TX>::type;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)nc * n) return;
    const int64_t I = g / n;
    const int q = (int)(g - I * n);
    A s = 0;
    for (int32_t m = aptr[I]; m < aptr[I + 1]; ++m) s += (A)r[(int64_t)amem[m] * n + q];
    bc[g] = (TX)s;
}

template <typename TX>
__global__ void k_prolong(int32_t N, int n, const int32_t *__restrict__ agg, const TX *__restrict__ e,
                          TX *__restrict__ x) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)N * n) return;
    const int64_t i = g / n;
    const int q = (int)(g - i * n);
    x[g] += e[(int64_t)agg[i] * n + q];
}

template <typename TA, typename TB>
__global__ void k_cast(int64_t m, const TA *__restrict__ a, TB *__restrict__ b) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < m) b[g] = (TB)a[g];
}

// Coarsest level: x_s = inv_s b_s for every system s (one workgroup each), FP64.
template <typename TX>
__global__ __launch_bounds__(256) void k_coarse(const double *__restrict__ inv, const int64_t *__restrict__ off,
                                                const int32_t *__restrict__ msz, const int64_t *__restrict__ roff,
                                                const TX *__restrict__ b, TX *__restrict__ x) {
    extern __shared__ double sb[];
    const int s = blockIdx.x;
    const int m = msz[s];
    const int64_t r0 = roff[s];
    for (int c = threadIdx.x; c < m; c += blockDim.x) sb[c] = (double)b[r0 + c];
    __syncthreads();
    const double *M = inv + off[s];
    for (int r = threadIdx.x; r < m; r += blockDim.x) {
        double acc = 0.0;
        for (int c = 0; c < m; ++c) acc += M[(int64_t)r * m + c] * sb[c];
        x[r0 + r] = (TX)acc;
    }
}

template <int n>
__global__ void k_block_apply(int32_t N, const double *__restrict__ Dinv, const double *__restrict__ r,
                              double *__restrict__ z) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)N * n) return;
    const int64_t i = g / n;
    const int q = (int)(g - i * n);
    const double *Di = Dinv + i * (n * n) + q * n;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < n; ++c) s += Di[c] * r[i * n + c];
    z[g] = s;
}

}  // namespace

template <typename TV, typename TX>
void launch_rows(int mode, int n, const SellView &S, const TV *val, const TX *x, const TX *b, TX *y,
                 const double *Dinv, double omega, hipStream_t st, TX *aux, const int32_t *pagg, const TX *pe,
                 double *y64) {
    if (S.N <= 0) return;
    switch (n) {
        case 1: rows_n<1>(mode, S, val, x, b, y, Dinv, omega, aux, pagg, pe, y64, st); break;
        case 2: rows_n<2>(mode, S, val, x, b, y, Dinv, omega, aux, pagg, pe, y64, st); break;
        case 3: rows_n<3>(mode, S, val, x, b, y, Dinv, omega, aux, pagg, pe, y64, st); break;
        case 4: rows_n<4>(mode, S, val, x, b, y, Dinv, omega, aux, pagg, pe, y64, st); break;
        case 5: rows_n<5>(mode, S, val, x, b, y, Dinv, omega, aux, pagg, pe, y64, st); break;
    }
    LAUNCHCHK();
}
template void launch_rows<double, double>(int, int, const SellView &, const double *, const double *, const double *,
                                          double *, const double *, double, hipStream_t, double *,
                                          const int32_t *, const double *, double *);
template void launch_rows<float, float>(int, int, const SellView &, const float *, const float *, const float *,
                                        float *, const double *, double, hipStream_t, float *, const int32_t *,
                                        const float *, double *);

void sell_pattern_begin(int32_t N, const int32_t *rp, const int32_t *col, Sell &S, hipStream_t st, bool offdiag,
                        int slice, const int32_t *rows_by_colour, const std::vector<int32_t> *colour_off) {
    int lc = 0;
    while ((1 << lc) < slice) ++lc;
    if ((1 << lc) != slice || lc > 6) cbs_throw(CBS_ERR_ARG, "slice height must be a power of two up to 64");
    const int32_t C = 1 << lc;
    S.N = N;
    S.lc = lc;
    if (rows_by_colour && colour_off) {
        const int ncol = (int)colour_off->size() - 1;
        if (ncol > kMaxColourRanges) cbs_throw(CBS_ERR_ARG, "too many colours");
        ColourRanges cr{};
        cr.ncol = ncol;
        S.cpos.assign(ncol + 1, 0);
        for (int c = 0; c <= ncol; ++c) {
            cr.off[c] = (*colour_off)[c];
            if (c > 0) {
                const int32_t cnt = (*colour_off)[c] - (*colour_off)[c - 1];
                S.cpos[c] = S.cpos[c - 1] + (cnt + C - 1) / C * C;
            }
            cr.cpos[c] = S.cpos[c];
        }
        S.npos = S.cpos[ncol];
        S.prow.alloc(S.npos > 0 ? S.npos : 1);
        if (S.npos > 0)
            hipLaunchKernelGGL(k_fill_i32, dim3(cdiv(S.npos, 256)), dim3(256), 0, st, (int64_t)S.npos, S.prow.get(), -1);
        if (N > 0)
            hipLaunchKernelGGL(k_colour_positions, dim3(cdiv(N, 256)), dim3(256), 0, st, N, cr, rows_by_colour,
                               S.prow.get());
    } else {
        S.prow.release();
        S.cpos.clear();
        S.npos = N;
    }
    S.nslices = (S.npos + C - 1) / C;
    const int32_t ns = S.nslices;
    S.sw.alloc(ns > 0 ? ns : 1);
    S.soff.alloc(ns + 1);
    if (ns > 0)
        hipLaunchKernelGGL(k_sell_width, dim3(cdiv((int64_t)ns * C, 256)), dim3(256), 0, st, S.npos, ns, C, rp, col,
                           S.prow.get(), S.sw.get(), S.soff.get(), offdiag ? 1 : 0);
    LAUNCHCHK();
    scan_exclusive(S.soff.get(), S.soff.get(), ns, st);
}

void sell_pattern_finish(const int32_t *rp, const int32_t *col, Sell &S, int64_t nent, hipStream_t st,
                         bool offdiag) {
    S.nent = nent;
    S.scol.alloc(S.nent > 0 ? S.nent : 1);
    S.ssrc.alloc(S.nent > 0 ? S.nent : 1);
    if (S.nent > 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(cdiv(S.nent, 256)), dim3(256), 0, st, S.nent, S.scol.get(), -1);
        hipLaunchKernelGGL(k_fill_i32, dim3(cdiv(S.nent, 256)), dim3(256), 0, st, S.nent, S.ssrc.get(), -1);
    }
    if (S.npos > 0)
        hipLaunchKernelGGL(k_sell_fill_idx, dim3(cdiv(S.npos, 256)), dim3(256), 0, st, S.npos, 1 << S.lc, rp, col,
                           S.prow.get(), S.soff.get(), S.scol.get(), S.ssrc.get(), offdiag ? 1 : 0);
    LAUNCHCHK();
}

void sell_build(int32_t N, const int32_t *rp, const int32_t *col, Sell &S, hipStream_t st, bool offdiag, int slice,
                const int32_t *rows_by_colour, const std::vector<int32_t> *colour_off) {
    sell_pattern_begin(N, rp, col, S, st, offdiag, slice, rows_by_colour, colour_off);
    sell_pattern_finish(rp, col, S, read_int(S.soff.get() + S.nslices, st), st, offdiag);
}

void sell_fill(int n, const Sell &S, const double *bcsr_vals, double *out, hipStream_t st, float *out32,
               int32_t *flag) {
    const int64_t tot = S.nent * n * n;
    if (tot <= 0) return;
    const dim3 b(256);
#define SV(NN)                                                                                                  \
    if (out32)                                                                                                  \
        hipLaunchKernelGGL((k_sell_vals<NN, true>), dim3(cdiv(tot / kSellV(NN), 256)), b, 0, st, S.nent,          \
                           S.ssrc.get(), bcsr_vals, out, out32, flag);                                          \
    else                                                                                                        \
        hipLaunchKernelGGL((k_sell_vals<NN, false>), dim3(cdiv(tot / kSellV(NN), 256)), b, 0, st, S.nent,         \
                           S.ssrc.get(), bcsr_vals, out, nullptr, nullptr)
    switch (n) {
        case 1: SV(1); break;
        case 2: SV(2); break;
        case 3: SV(3); break;
        case 4: SV(4); break;
        case 5: SV(5); break;
    }
#undef SV
    LAUNCHCHK();
}

void sell_fill_scaled(int n, const Sell &F, const Sell &O, const double *bcsr_vals, const double *Dinv,
                      double *f64, float *f32, float *o32, int32_t *flag, hipStream_t st) {
    if (F.N <= 0) return;
    if (F.lc != O.lc || F.nslices != O.nslices || F.prow.get() || O.prow.get())
        cbs_throw(CBS_ERR_ARG, "sliced copies do not share their slices");
    const int64_t npos = (int64_t)F.nslices << F.lc;
    const dim3 g(cdiv(npos, 64));
#define FS_N(NN)                                                                                               \
    hipLaunchKernelGGL(k_sell_fill_scaled<NN>, g, dim3(64 * NN), 0, st, F.N, F.nslices, F.lc, F.soff.get(),     \
                       F.sw.get(), F.scol.get(), F.ssrc.get(), O.soff.get(), O.sw.get(), bcsr_vals, Dinv, f64, \
                       f32, o32, flag)
    switch (n) {
        case 1: FS_N(1); break;
        case 2: FS_N(2); break;
        case 3: FS_N(3); break;
        case 4: FS_N(4); break;
        case 5: FS_N(5); break;
    }
#undef FS_N
    LAUNCHCHK();
}

void sell_scale(int n, const Sell &S, const double *bcsr_vals, const double *Dinv, float *out, int32_t *flag,
                hipStream_t st) {
    const int64_t npos = (int64_t)S.nslices << S.lc;
    if (S.N <= 0) return;
    const dim3 g(cdiv(npos, 64));
#define SCALE_N(NN)                                                                                           \
    hipLaunchKernelGGL(k_sell_scaled<NN>, g, dim3(64 * NN), 0, st, S.N, S.nslices, S.lc, S.soff.get(), S.sw.get(), \
                       S.ssrc.get(), bcsr_vals, Dinv, out, flag)
    switch (n) {
        case 1: SCALE_N(1); break;
        case 2: SCALE_N(2); break;
        case 3: SCALE_N(3); break;
        case 4: SCALE_N(4); break;
        case 5: SCALE_N(5); break;
    }
#undef SCALE_N
    LAUNCHCHK();
}

template <int n, typename TX>
__global__ __launch_bounds__(64 * n) void k_restrict_sweep0(int32_t nc, const int32_t *__restrict__ aptr,
                                                            const int32_t *__restrict__ amem,
                                                            const TX *__restrict__ r, TX *__restrict__ b,
                                                            const double *__restrict__ Dinv, double omega,
                                                            TX *__restrict__ x, TX *__restrict__ c) {
    using A = typename Acc<TX>::type;
    constexpr int nn = n * n;
    const int t = threadIdx.x;
    const int lr = t / n, q = t - lr * n;
    const int32_t I = blockIdx.x * 64 + lr;
    A s = 0;
    if (I < nc)
        for (int32_t m = aptr[I]; m < aptr[I + 1]; ++m) s += (A)r[(int64_t)amem[m] * n + q];
    const TX bv = (TX)s;
    const int64_t o = (int64_t)I * n + q;
    if (I < nc) b[o] = bv;
    __shared__ A sb[64 * n];
    sb[t] = (A)bv;
    __syncthreads();
    if (I < nc) {
        const double *Di = Dinv + (int64_t)I * nn + q * n;
        double z = 0.0;
#pragma unroll
        for (int k = 0; k < n; ++k) z += Di[k] * (double)sb[lr * n + k];
        x[o] = (TX)((A)0 + (A)(omega * z));
        if (c) c[o] = (TX)z;
    }
}

// Mixed precision, level 0: the FP64 right side rounded to FP32 (kept in b
// for the residual) fused with the zero-guess sweep x = omega Dinv b,
// c = Dinv b.  Same roundings as a cast kernel followed by mode 3.
template <int n>
__global__ __launch_bounds__(64 * n) void k_cast_sweep0(int32_t N, const double *__restrict__ b64,
                                                        float *__restrict__ b, const double *__restrict__ Dinv,
                                                        double omega, float *__restrict__ x, float *__restrict__ c) {
    constexpr int nn = n * n;
    const int t = threadIdx.x;
    const int lr = t / n, q = t - lr * n;
    const int32_t i = blockIdx.x * 64 + lr;
    const int64_t o = (int64_t)i * n + q;
    const float bv = i < N ? (float)b64[o] : 0.0f;
    if (i < N) b[o] = bv;
    __shared__ float sb[64 * n];
    sb[t] = bv;
    __syncthreads();
    if (i < N) {
        const double *Di = Dinv + (int64_t)i * nn + q * n;
        double z = 0.0;
#pragma unroll
        for (int k = 0; k < n; ++k) z += Di[k] * (double)sb[lr * n + k];
        x[o] = (float)(0.0f + (float)(omega * z));
        if (c) c[o] = (float)z;
    }
}

void launch_cast_sweep0(int n, int32_t N, const double *b64, float *b, const double *Dinv, double omega, float *x,
                        float *c, hipStream_t st) {
    if (N <= 0) return;
    const dim3 g(cdiv(N, 64)), bl(64 * n);
#define CS0(NN) hipLaunchKernelGGL((k_cast_sweep0<NN>), g, bl, 0, st, N, b64, b, Dinv, omega, x, c)
    switch (n) {
        case 1: CS0(1); break;
        case 2: CS0(2); break;
        case 3: CS0(3); break;
        case 4: CS0(4); break;
        case 5: CS0(5); break;
    }
#undef CS0
    LAUNCHCHK();
}

template <typename TX>
void launch_restrict_sweep0(int n, int32_t nc, const int32_t *agg_ptr, const int32_t *agg_mem, const TX *r, TX *b,
                            const double *Dinv, double omega, TX *x, TX *c, hipStream_t st) {
    if (nc <= 0) return;
    const dim3 g(cdiv(nc, 64)), bl(64 * n);
#define RS0(NN) hipLaunchKernelGGL((k_restrict_sweep0<NN, TX>), g, bl, 0, st, nc, agg_ptr, agg_mem, r, b, Dinv, omega, x, c)
    switch (n) {
        case 1: RS0(1); break;
        case 2: RS0(2); break;
        case 3: RS0(3); break;
        case 4: RS0(4); break;
        case 5: RS0(5); break;
    }
#undef RS0
    LAUNCHCHK();
}
template void launch_restrict_sweep0<double>(int, int32_t, const int32_t *, const int32_t *, const double *, double *,
                                             const double *, double, double *, double *, hipStream_t);
template void launch_restrict_sweep0<float>(int, int32_t, const int32_t *, const int32_t *, const float *, float *,
                                            const double *, double, float *, float *, hipStream_t);

template <typename TX>
void launch_restrict(int n, int32_t nc, const int32_t *agg_ptr, const int32_t *agg_mem, const TX *r, TX *bc,
                     hipStream_t st) {
    const int64_t m = (int64_t)nc * n;
    if (m > 0) hipLaunchKernelGGL(k_restrict<TX>, dim3(cdiv(m, 256)), dim3(256), 0, st, nc, n, agg_ptr, agg_mem, r, bc);
    LAUNCHCHK();
}
template void launch_restrict<double>(int, int32_t, const int32_t *, const int32_t *, const double *, double *, hipStream_t);
template void launch_restrict<float>(int, int32_t, const int32_t *, const int32_t *, const float *, float *, hipStream_t);

template <typename TX>
void launch_prolong(int n, int32_t N, const int32_t *agg, const TX *e, TX *x, hipStream_t st) {
    const int64_t m = (int64_t)N * n;
    if (m > 0) hipLaunchKernelGGL(k_prolong<TX>, dim3(cdiv(m, 256)), dim3(256), 0, st, N, n, agg, e, x);
    LAUNCHCHK();
}
template void launch_prolong<double>(int, int32_t, const int32_t *, const double *, double *, hipStream_t);
template void launch_prolong<float>(int, int32_t, const int32_t *, const float *, float *, hipStream_t);

namespace {
template <typename T>
__global__ void k_fill0(int64_t m, T *a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < m) a[g] = (T)0;
}
}  // namespace

void launch_copy(int64_t m, const double *a, double *b, hipStream_t st) {
    if (m > 0) hipLaunchKernelGGL((k_cast<double, double>), dim3(cdiv(m, 256)), dim3(256), 0, st, m, a, b);
    LAUNCHCHK();
}

template <typename T>
void launch_fill(int64_t m, T *a, hipStream_t st) {
    if (m > 0) hipLaunchKernelGGL(k_fill0<T>, dim3(cdiv(m, 256)), dim3(256), 0, st, m, a);
    LAUNCHCHK();
}
template void launch_fill<double>(int64_t, double *, hipStream_t);
template void launch_fill<float>(int64_t, float *, hipStream_t);

template <typename TA, typename TB>
void launch_cast(int64_t m, const TA *a, TB *b, hipStream_t st) {
    if (m > 0) hipLaunchKernelGGL((k_cast<TA, TB>), dim3(cdiv(m, 256)), dim3(256), 0, st, m, a, b);
    LAUNCHCHK();
}
template void launch_cast<double, float>(int64_t, const double *, float *, hipStream_t);
template void launch_cast<float, double>(int64_t, const float *, double *, hipStream_t);
template void launch_cast<double, double>(int64_t, const double *, double *, hipStream_t);
template void launch_cast<float, float>(int64_t, const float *, float *, hipStream_t);

void launch_coarse_solve(cbs_system *h, bool transposed, const void *b, void *x, bool fp32) {
    Coarse &C = h->coarse;
    const double *inv = transposed ? C.invT.get() : C.inv.get();
    const size_t shm = sizeof(double) * (size_t)C.max_m;
    if (fp32)
        hipLaunchKernelGGL(k_coarse<float>, dim3(h->n_sys), dim3(256), shm, h->stream, inv, C.off.get(), C.m.get(),
                           C.roff.get(), (const float *)b, (float *)x);
    else
        hipLaunchKernelGGL(k_coarse<double>, dim3(h->n_sys), dim3(256), shm, h->stream, inv, C.off.get(), C.m.get(),
                           C.roff.get(), (const double *)b, (double *)x);
    LAUNCHCHK();
}

void launch_block_apply(int n, int32_t N, const double *Dinv, const double *r, double *z, hipStream_t st) {
    const int64_t m = (int64_t)N * n;
    if (m <= 0) return;
    const dim3 g(cdiv(m, 256)), b(256);
    switch (n) {
        case 1: hipLaunchKernelGGL(k_block_apply<1>, g, b, 0, st, N, Dinv, r, z); break;
        case 2: hipLaunchKernelGGL(k_block_apply<2>, g, b, 0, st, N, Dinv, r, z); break;
        case 3: hipLaunchKernelGGL(k_block_apply<3>, g, b, 0, st, N, Dinv, r, z); break;
        case 4: hipLaunchKernelGGL(k_block_apply<4>, g, b, 0, st, N, Dinv, r, z); break;
        case 5: hipLaunchKernelGGL(k_block_apply<5>, g, b, 0, st, N, Dinv, r, z); break;
    }
    LAUNCHCHK();
}

template <typename T>
void launch_gs_colour(int n, const SellView &S, const T *val, int32_t p0, int32_t cnt, const double *Dinv,
                      const T *b, T *x, hipStream_t st, int form, T *rz) {
    if (cnt <= 0) return;
    if (form < 0 || form > 2) cbs_throw(CBS_ERR_ARG, "Gauss-Seidel colour step: bad form");
    const dim3 g(cdiv(cnt, 64));
#define GS_F(NN, FF) hipLaunchKernelGGL((k_gs_colour<NN, T, FF>), g, dim3(64 * NN), 0, st, S, val, p0, cnt, Dinv, b, x, rz)
#define GS_C(NN)                      \
    {                                 \
        if (form == 0) GS_F(NN, 0);   \
        else if (form == 1) GS_F(NN, 1); \
        else GS_F(NN, 2);             \
    }
    switch (n) {
        case 1: GS_C(1); break;
        case 2: GS_C(2); break;
        case 3: GS_C(3); break;
        case 4: GS_C(4); break;
        case 5: GS_C(5); break;
    }
#undef GS_C
#undef GS_F
    LAUNCHCHK();
}
template void launch_gs_colour<double>(int, const SellView &, const double *, int32_t, int32_t, const double *,
                                       const double *, double *, hipStream_t, int, double *);
template void launch_gs_colour<float>(int, const SellView &, const float *, int32_t, int32_t, const double *,
                                      const float *, float *, hipStream_t, int, float *);

template <typename T>
void launch_dilu_fwd(int n, const SellView &S, const T *val, const T *fval, const int32_t *colour, int c, int32_t p0,
                     int32_t cnt, const double *Einv, const T *b, T *x, T *y, bool zero_guess, bool last,
                     hipStream_t st) {
    if (cnt <= 0) return;
    const dim3 g(cdiv(cnt, 64));
    if (zero_guess && fval) {                  // no residual: only the factor is read
        val = fval;
        fval = nullptr;
    }
#define DILU_F1(NN, Z, LA)                                                                                       \
    hipLaunchKernelGGL((k_dilu_fwd<NN, T, Z, LA>), g, dim3(64 * NN), 0, st, S, val, fval, colour, c, p0, cnt, Einv, \
                       b, x, y)
#define DILU_F(NN)                                                                                               \
    if (zero_guess) { if (last) DILU_F1(NN, true, true); else DILU_F1(NN, true, false); }                         \
    else { if (last) DILU_F1(NN, false, true); else DILU_F1(NN, false, false); }
    switch (n) {
        case 1: DILU_F(1) break;
        case 2: DILU_F(2) break;
        case 3: DILU_F(3) break;
        case 4: DILU_F(4) break;
        case 5: DILU_F(5) break;
    }
#undef DILU_F
#undef DILU_F1
    LAUNCHCHK();
}

template <typename T>
void launch_dilu_bwd(int n, const SellView &S, const T *val, const int32_t *colour, int c, int32_t p0, int32_t cnt,
                     const double *Einv, T *yz, T *x, bool zero_guess, hipStream_t st) {
    if (cnt <= 0) return;
    const dim3 g(cdiv(cnt, 64));
#define DILU_B(NN)                                                                                              \
    if (zero_guess)                                                                                             \
        hipLaunchKernelGGL((k_dilu_bwd<NN, T, true>), g, dim3(64 * NN), 0, st, S, val, colour, c, p0, cnt, Einv, yz, x); \
    else                                                                                                        \
        hipLaunchKernelGGL((k_dilu_bwd<NN, T, false>), g, dim3(64 * NN), 0, st, S, val, colour, c, p0, cnt, Einv, yz, x);
    switch (n) {
        case 1: DILU_B(1) break;
        case 2: DILU_B(2) break;
        case 3: DILU_B(3) break;
        case 4: DILU_B(4) break;
        case 5: DILU_B(5) break;
    }
#undef DILU_B
    LAUNCHCHK();
}

template void launch_dilu_fwd<double>(int, const SellView &, const double *, const double *, const int32_t *, int,
                                      int32_t, int32_t, const double *, const double *, double *, double *, bool, bool,
                                      hipStream_t);
template void launch_dilu_fwd<float>(int, const SellView &, const float *, const float *, const int32_t *, int,
                                     int32_t, int32_t, const double *, const float *, float *, float *, bool, bool,
                                     hipStream_t);
template void launch_dilu_bwd<double>(int, const SellView &, const double *, const int32_t *, int, int32_t, int32_t,
                                      const double *, double *, double *, bool, hipStream_t);
template void launch_dilu_bwd<float>(int, const SellView &, const float *, const int32_t *, int, int32_t, int32_t,
                                     const double *, float *, float *, bool, hipStream_t);

// ------------------------------------------------------------------ autotuning
// The residual kernel (the shape shared by SpMV and the smoother sweeps) is
// timed with HIP events for each schedule on the matrix itself; the fastest
// is kept per (rows, entries, block size, precision) for the process.
namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int32_t, int64_t, int, bool>, Sched> g_tune_cache;
}  // namespace

// Levels of fewer than kSplitLevelRows block rows split each row over several
// threads; automatic choice from the mean row length (nblocks / N, stored
// blocks only): the largest power of two (at most 16) that still leaves every
// thread about three blocks.  (Level 2 of the 1M-cell p-U system, 47,807
// rows, runs its sweep in 13.1 us with one thread per scalar row against
// 14.1 us split four ways.)
int8_t row_split_for(const Sell &S, int64_t nblocks, int32_t opt_split) {
    if (S.N <= 0 || S.N >= kSplitLevelRows) return 1;
    if (opt_split > 0) return (int8_t)opt_split;
    const double w = (double)nblocks / S.N;
    int s = 1;
    while (s < 16 && 3.0 * (2 * s) <= w) s *= 2;
    return (int8_t)s;
}

Sched choose_sched(int n, const Sell &S, bool fp32, const void *val, int32_t forced, hipStream_t st) {
    if (forced >= 1 && forced <= 6) {
        static const int8_t unroll[3] = {1, 2, 4};
        return Sched{unroll[(forced - 1) / 2], (int8_t)((forced - 1) % 2)};
    }
    return autotune_rows(n, S, fp32, val, st);
}

Sched autotune_rows(int n, const Sell &S, bool fp32, const void *val, hipStream_t st) {
    const auto key = std::make_tuple(S.N, S.nent, n, fp32);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) return it->second;
    }
    Sched best = fp32 ? Sched{4, 1} : Sched{4, 0};
    if (S.N < 65536) return best;                        // small levels: launch-bound, keep the default
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // the default is kept unless another variant is clearly (3%) faster, so
    // that near-ties do not flip the choice from one run to the next
    const Sched dflt = best;
    float best_ms = 1e30f, dflt_ms = 1e30f;
    const int64_t m = (int64_t)S.N * n;
    DArr<double> scratch((size_t)3 * m);
    void *x = scratch.get(), *b = scratch.get() + m, *y = scratch.get() + 2 * m;
    if (fp32) { launch_fill<float>(m, (float *)x, st); launch_fill<float>(m, (float *)b, st); }
    else { launch_fill<double>(m, (double *)x, st); launch_fill<double>(m, (double *)b, st); }
    // three rounds over the six variants, each variant's best round kept:
    // drifts of the clock or of other work affect every variant alike
    float vms[6];
    for (float &t : vms) t = 1e30f;
    for (int round = 0; round < 3; ++round)
        for (int vi = 0; vi < 6; ++vi) {
            SellView v = S.view(fp32);
            v.sched = Sched{(int8_t)(vi < 2 ? 1 : (vi < 4 ? 2 : 4)), (int8_t)(vi & 1)};
            auto run = [&] {
                if (fp32)
                    launch_rows<float, float>(1, n, v, (const float *)val, (const float *)x, (const float *)b, (float *)y,
                                              nullptr, 0.0, st);
                else
                    launch_rows<double, double>(1, n, v, (const double *)val, (const double *)x, (const double *)b,
                                                (double *)y, nullptr, 0.0, st);
            };
            run();
            HIPCHK(hipEventRecord(e0, st));
            for (int rep = 0; rep < 3; ++rep) run();
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            vms[vi] = std::min(vms[vi], ms);
        }
    for (int vi = 0; vi < 6; ++vi) {
        const Sched sv{(int8_t)(vi < 2 ? 1 : (vi < 4 ? 2 : 4)), (int8_t)(vi & 1)};
        if (sv.unroll == dflt.unroll && sv.nontemporal == dflt.nontemporal) dflt_ms = vms[vi];
        if (vms[vi] < best_ms) { best_ms = vms[vi]; best = sv; }
    }
    if (best_ms > 0.97f * dflt_ms) best = dflt;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
    return best;
}
