// krylov.hip -- preconditioned BiCGStab and flexible GMRES(m) on the device,
// the AMG V-cycle, and the mixed-precision wrapper.
//
// Solver families of Sec. 2.3 (GMRES, bi-conjugate gradient) with the AMG
// preconditioner.  All Krylov scalars (rho, alpha, omega, Hessenberg, Givens)
// live in device memory, one set per system, so a batch of independent
// systems runs through the same launches; the host only reads the
// per-system "converged" flags every `check_every` iterations.  Reductions
// are two-stage and deterministic: one partial per (system, work item),
// then a per-system sum over its items in a fixed order.
//
// Mixed precision: the hierarchy (level matrices, smoother sweeps, level
// vectors) runs in FP32, while residuals, inner products, D^{-1} and the
// coarsest dense inverse stay FP64 (FP64 -> FP32 casts round to nearest even).
#include "cbs_internal.h"

#include <algorithm>
#include <cmath>

namespace {

enum { PH_INIT = 0, PH_ALPHA, PH_OMEGA, PH_END, PH_RESTART, PH_TRUE, PH_SNORM };

// flags bits: 1 breakdown; 2 converged at the half step (||s|| met the
// tolerance: the iteration ends with x += alpha ph, r = s); 4 the residual,
// shrinking as in the last iteration, would be within 4x of the tolerance
// after the next one
constexpr int32_t kFlagBreak = 1, kFlagHalf = 2, kFlagNear = 4;
// partial sums of (s, s), written with s, read at the half-step test
constexpr int kSlotSS = 2;

__device__ inline double block_sum(double v, double *sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    __syncthreads();
    return t;   // valid in thread 0
}

// up to three dot products of one work item -> partial[q * n_items + item]
__global__ __launch_bounds__(kVecThreads) void k_dots(const Item *__restrict__ items, int32_t n_items,
                                                      const int32_t *__restrict__ done, int K,
                                                      const double *a0, const double *b0, const double *a1,
                                                      const double *b1, const double *a2, const double *b2,
                                                      double *partial) {
    __shared__ double sh[kVecThreads / 64];
    const Item it = items[blockIdx.x];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (!done[it.sys]) {
        for (int64_t e = it.beg + threadIdx.x; e < it.end; e += kVecThreads) {
            s0 += a0[e] * b0[e];
            if (K > 1) s1 += a1[e] * b1[e];
            if (K > 2) s2 += a2[e] * b2[e];
        }
    }
    s0 = block_sum(s0, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s0;
    if (K > 1) { s1 = block_sum(s1, sh); if (threadIdx.x == 0) partial[n_items + blockIdx.x] = s1; }
    if (K > 2) { s2 = block_sum(s2, sh); if (threadIdx.x == 0) partial[2 * n_items + blockIdx.x] = s2; }
}

// Sum of one system's partials, by the whole workgroup: thread t adds items
// i0+t, i0+t+256, ... in order, then a fixed tree combines the threads, so
// the result does not depend on timing.  Every thread gets the value.
constexpr int kFinThreads = 256;

__device__ inline double sum_items(const double *partial, int32_t n_items, int q, int32_t i0, int32_t i1) {
    __shared__ double sh[kFinThreads / 64];
    __shared__ double res;
    double t = 0.0;
    for (int32_t k = i0 + (int32_t)threadIdx.x; k < i1; k += kFinThreads) t += partial[(int64_t)q * n_items + k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
        for (int w = 0; w < kFinThreads / 64; ++w) a += sh[w];
        res = a;
    }
    __syncthreads();
    const double v = res;
    __syncthreads();
    return v;
}

#define SC(slot) scal[(slot) * nsys + s]

// Per-system scalar updates after a reduction.
__global__ __launch_bounds__(kFinThreads) void k_fin(int phase, int32_t nsys, const int32_t *__restrict__ item_off,
                                                      int32_t n_items, const double *__restrict__ partial, double *scal,
                                                      int32_t *done, int32_t *flags, int32_t *iters, double tol2,
                                                      const int32_t *restart_mask) {
    const int s = blockIdx.x;
    const int32_t i0 = item_off[s], i1 = item_off[s + 1];
    // every phase needs at most two sums; compute them with the whole group
    const bool skip = (phase == PH_RESTART && !restart_mask[s]) ||
                      ((phase == PH_ALPHA || phase == PH_OMEGA || phase == PH_END || phase == PH_SNORM) &&
                       (done[s] || (flags[s] & kFlagBreak)));
    if (skip) return;
    const double q0 = phase == PH_SNORM ? 0.0 : sum_items(partial, n_items, 0, i0, i1);
    const double q1 = (phase == PH_INIT || phase == PH_OMEGA || phase == PH_END) ? sum_items(partial, n_items, 1, i0, i1)
                                                                                 : 0.0;
    const double qss = (phase == PH_SNORM || phase == PH_OMEGA) ? sum_items(partial, n_items, kSlotSS, i0, i1) : 0.0;
    if (threadIdx.x != 0) return;
    if (phase == PH_INIT) {
        const double rr = q0, bb = q1;
        SC(S_RR) = rr; SC(S_BB) = bb; SC(S_RES0) = bb > 0.0 ? sqrt(rr / bb) : 0.0;
        SC(S_RHO) = rr; SC(S_RHO0) = 1.0; SC(S_ALPHA) = 1.0; SC(S_OMEGA) = 1.0; SC(S_RRPREV) = 0.0;
        done[s] = (bb == 0.0 || rr <= tol2 * bb) ? 1 : 0;
        flags[s] = 0;
        iters[s] = 0;
        return;
    }
    if (phase == PH_TRUE) {                          // true residual of every system
        SC(S_RR) = q0;
        return;
    }
    if (phase == PH_RESTART) {                       // rhat = r; p = v = 0 done by the caller
        const double rr = q0;
        SC(S_RR) = rr; SC(S_RHO) = rr; SC(S_RHO0) = 1.0; SC(S_ALPHA) = 1.0; SC(S_OMEGA) = 1.0;
        SC(S_RRPREV) = 0.0;
        done[s] = (SC(S_BB) == 0.0 || rr <= tol2 * SC(S_BB)) ? 1 : 0;
        flags[s] = 0;
        return;
    }
    if (phase == PH_ALPHA) {
        const double rv = q0;
        SC(S_RV) = rv;
        const double rho = SC(S_RHO);
        if (rv == 0.0 || !isfinite(rv) || fabs(rv) < 1e-300 * fmax(SC(S_RR), 1e-300)) {
            flags[s] |= 1;
            SC(S_ALPHA) = 0.0;
        } else {
            SC(S_ALPHA) = rho / rv;
        }
        iters[s] += 1;
    } else if (phase == PH_SNORM) {                  // ||s||^2: converged at the half step?
        if (qss <= tol2 * SC(S_BB)) flags[s] |= kFlagHalf;
    } else if (phase == PH_OMEGA) {
        if (qss <= tol2 * SC(S_BB)) flags[s] |= kFlagHalf;
        const double ts = q0, tt = q1;
        SC(S_TS) = ts; SC(S_TT) = tt;
        SC(S_OMEGA) = (flags[s] & kFlagHalf) ? 0.0 : (tt > 0.0 ? ts / tt : 0.0);
    } else if (phase == PH_END) {
        const double rr = q0, rhn = q1;
        SC(S_RR) = rr;
        SC(S_RHO0) = SC(S_RHO);
        SC(S_RHO) = rhn;
        if (rr <= tol2 * SC(S_BB)) done[s] = 1;
        else if (SC(S_OMEGA) == 0.0 || rhn == 0.0 || !isfinite(rhn) || (flags[s] & kFlagBreak)) flags[s] |= kFlagBreak;
        flags[s] &= ~(kFlagHalf | kFlagNear);
        const double rrp = SC(S_RRPREV);
        if (rrp > 0.0 && rr * (rr / rrp) <= 16.0 * tol2 * SC(S_BB)) flags[s] |= kFlagNear;
        SC(S_RRPREV) = rr;
    }
}

// p = r + beta (p - omega v),  beta = (rho / rho0) (alpha / omega)
__global__ __launch_bounds__(kVecThreads) void k_p_update(const Item *__restrict__ items, int32_t nsys,
                                                          const int32_t *__restrict__ done,
                                                          const double *__restrict__ scal,
                                                          const int32_t *__restrict__ flags, const double *r,
                                                          double *p, const double *v) {
    const Item it = items[blockIdx.x];
    const int s = it.sys;
    if (done[s] || (flags[s] & kFlagBreak)) return;
    const double omega = SC(S_OMEGA);
    const double beta = (SC(S_RHO) / SC(S_RHO0)) * (SC(S_ALPHA) / omega);
    for (int64_t e = it.beg + threadIdx.x; e < it.end; e += kVecThreads) p[e] = r[e] + beta * (p[e] - omega * v[e]);
}

// s = r - alpha v, and partials of (s, s) for the half-step test
__global__ __launch_bounds__(kVecThreads) void k_s_update(const Item *__restrict__ items, int32_t n_items,
                                                          int32_t nsys, const int32_t *__restrict__ done,
                                                          const double *__restrict__ scal,
                                                          const int32_t *__restrict__ flags, const double *r,
                                                          const double *v, double *sv, double *partial) {
    __shared__ double red[kVecThreads / 64];
    const Item it = items[blockIdx.x];
    const int s = it.sys;
    double s0 = 0.0;
    if (!done[s] && !(flags[s] & kFlagBreak)) {
        const double alpha = SC(S_ALPHA);
        for (int64_t e = it.beg + threadIdx.x; e < it.end; e += kVecThreads) {
            const double se = r[e] - alpha * v[e];
            sv[e] = se;
            s0 += se * se;
        }
    }
    s0 = block_sum(s0, red);
    if (threadIdx.x == 0) partial[(int64_t)kSlotSS * n_items + blockIdx.x] = s0;
}

// x += alpha ph + omega sh;  r = s - omega t;  partials (r,r), (rhat,r).
// A system converged at the half step takes x += alpha ph, r = s.
__global__ __launch_bounds__(kVecThreads) void k_xr_update(const Item *__restrict__ items, int32_t n_items,
                                                           int32_t nsys, const int32_t *__restrict__ done,
                                                           const double *__restrict__ scal,
                                                           const int32_t *__restrict__ flags, double *x,
                                                           const double *ph, const double *sh, double *r,
                                                           const double *sv, const double *t, const double *rh,
                                                           double *partial) {
    __shared__ double red[kVecThreads / 64];
    const Item it = items[blockIdx.x];
    const int s = it.sys;
    double s0 = 0.0, s1 = 0.0;
    if (!done[s] && !(flags[s] & kFlagBreak)) {
        const double alpha = SC(S_ALPHA), omega = SC(S_OMEGA);
        if (flags[s] & kFlagHalf) {
            for (int64_t e = it.beg + threadIdx.x; e < it.end; e += kVecThreads) {
                x[e] += alpha * ph[e];
                const double re = sv[e];
                r[e] = re;
                s0 += re * re;
                s1 += rh[e] * re;
            }
        } else {
            for (int64_t e = it.beg + threadIdx.x; e < it.end; e += kVecThreads) {
                x[e] += alpha * ph[e] + omega * sh[e];
                const double re = sv[e] - omega * t[e];
                r[e] = re;
                s0 += re * re;
                s1 += rh[e] * re;
            }
        }
    }
    s0 = block_sum(s0, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s0;
    s1 = block_sum(s1, red);
    if (threadIdx.x == 0) partial[n_items + blockIdx.x] = s1;
}

// masked vector ops: y = a (copy), y = 0, x = 0 where b = 0 systems
__global__ void k_mask_copy(const Item *__restrict__ items, const int32_t *__restrict__ mask, int want,
                            const double *a, double *y) {
    const Item it = items[blockIdx.x];
    if ((mask[it.sys] != 0) != (want != 0)) return;
    for (int64_t e = it.beg + threadIdx.x; e < it.end; e += kVecThreads) y[e] = a ? a[e] : 0.0;
}

__global__ void k_zero_if_bzero(const Item *__restrict__ items, int32_t nsys, const double *__restrict__ scal,
                                double *x) {
    const Item it = items[blockIdx.x];
    const int s = it.sys;
    if (SC(S_BB) != 0.0) return;
    for (int64_t e = it.beg + threadIdx.x; e < it.end; e += kVecThreads) x[e] = 0.0;
}

// x += z (every element; a system that did not move contributes z = 0)
__global__ void k_gm_add(const Item *__restrict__ items, const double *__restrict__ z, double *x) {
    const Item it = items[blockIdx.x];
    for (int64_t e = it.beg + threadIdx.x; e < it.end; e += kVecThreads) x[e] += z[e];
}

// ------------------------------------------------------------------ FGMRES
// multi-dot: partial[i * n_items + item] = (w, V_i), i = 0..j
// partials of (V_i, w), i = 0..j; with ww also (w, w) in slot j + 1
__global__ __launch_bounds__(kVecThreads) void k_mdot(const Item *__restrict__ items, int32_t n_items,
                                                      const int32_t *__restrict__ done, int j, int64_t ld,
                                                      const double *__restrict__ V, const double *__restrict__ w,
                                                      double *partial, int ww) {
    __shared__ double red[kVecThreads / 64];
    const Item it = items[blockIdx.x];
    const bool act = !done[it.sys];
    for (int i = 0; i <= j + (ww ? 1 : 0); ++i) {
        const double *vi = i <= j ? V + i * ld : w;
        double acc = 0.0;
        if (act)
            for (int64_t e = it.beg + threadIdx.x; e < it.end; e += kVecThreads) acc += w[e] * vi[e];
        acc = block_sum(acc, red);
        if (threadIdx.x == 0) partial[(int64_t)i * n_items + blockIdx.x] = acc;
    }
}

// h_i (per system) = sum of partials; accumulate into H(:, j); store in coef.
// With skip (first pass, which also summed (w, w) in slot j + 1): a system
// whose w keeps more than a tenth of its norm, ||w - sum h_i V_i||^2 =
// ||w||^2 - sum h_i^2 > 0.01 ||w||^2, skips the second (re-orthogonalising)
// pass: skip[s] = 1 (also for a finished system).
__global__ __launch_bounds__(kFinThreads) void k_mdot_fin(int j, int m,
                                                           const int32_t *__restrict__ item_off, int32_t n_items,
                                                           const double *__restrict__ partial,
                                                           const int32_t *__restrict__ done, double *H, double *coef,
                                                           int accumulate, int32_t *skip) {
    const int s = blockIdx.x;
    if (done[s]) {
        if (skip && threadIdx.x == 0) skip[s] = 1;
        return;
    }
    double hh = 0.0;
    for (int i = 0; i <= j; ++i) {
        const double hv = sum_items(partial, n_items, i, item_off[s], item_off[s + 1]);
        hh += hv * hv;
        if (threadIdx.x == 0) {
            double *Hs = H + (int64_t)s * (m + 1) * m;
            Hs[i * m + j] = accumulate ? Hs[i * m + j] + hv : hv;
            coef[(int64_t)s * (m + 1) + i] = hv;
        }
    }
    if (skip) {
        const double ww = sum_items(partial, n_items, j + 1, item_off[s], item_off[s + 1]);
        if (threadIdx.x == 0) skip[s] = (ww - hh > 0.01 * ww) ? 1 : 0;
    }
}

// w -= sum_i coef_i V_i
__global__ __launch_bounds__(kVecThreads) void k_maxpy(const Item *__restrict__ items, const int32_t *__restrict__ done,
                                                       int j, int m, int64_t ld, const double *__restrict__ V,
                                                       const double *__restrict__ coef, double *w) {
    const Item it = items[blockIdx.x];
    if (done[it.sys]) return;
    const double *c = coef + (int64_t)it.sys * (m + 1);
    for (int64_t e = it.beg + threadIdx.x; e < it.end; e += kVecThreads) {
        double acc = w[e];
        for (int i = 0; i <= j; ++i) acc -= c[i] * V[i * ld + e];
        w[e] = acc;
    }
}

// y = a * inv(scal) per system: V_{j+1} = w / hn ; V_0 = r / beta
__global__ __launch_bounds__(kVecThreads) void k_scale(const Item *__restrict__ items, const int32_t *__restrict__ done,
                                                       const double *__restrict__ nrm, int stride, const double *a,
                                                       double *y) {
    const Item it = items[blockIdx.x];
    if (done[it.sys]) return;
    const double d = nrm[(int64_t)it.sys * stride];
    const double f = d > 0.0 ? 1.0 / d : 0.0;
    for (int64_t e = it.beg + threadIdx.x; e < it.end; e += kVecThreads) y[e] = a[e] * f;
}

// Restart start: beta = ||r||, g = (beta, 0, ...), converged check.
__global__ __launch_bounds__(kFinThreads) void k_gm_start(int32_t nsys, int m, const int32_t *__restrict__ item_off,
                                                           int32_t n_items, const double *__restrict__ partial,
                                                           double *scal, double *g, int32_t *done, int32_t *jlen,
                                                           double tol2, int first) {
    const int s = blockIdx.x;
    const double rr = sum_items(partial, n_items, 0, item_off[s], item_off[s + 1]);
    const double bbs = first ? sum_items(partial, n_items, 1, item_off[s], item_off[s + 1]) : 0.0;
    if (threadIdx.x != 0) return;
    SC(S_RR) = rr;
    if (first) {
        const double bb = bbs;
        SC(S_BB) = bb;
        SC(S_RES0) = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    }
    const double beta = sqrt(rr);
    SC(S_RHO) = beta;            // ||r|| of this cycle
    double *gs = g + (int64_t)s * (m + 1);
    for (int i = 0; i <= m; ++i) gs[i] = 0.0;
    gs[0] = beta;
    jlen[s] = 0;
    done[s] = (SC(S_BB) == 0.0 || rr <= tol2 * SC(S_BB)) ? 1 : 0;
}

// After the orthogonalisation of column j: H(j+1,j) = ||w||, apply the
// previous rotations, make rotation j, update g, and test |g(j+1)|.
__global__ __launch_bounds__(kFinThreads) void k_gm_givens(int32_t nsys, int j, int m,
                                                            const int32_t *__restrict__ item_off, int32_t n_items,
                                                            const double *__restrict__ partial, double *scal, double *H,
                                                            double *cs, double *sn, double *g, int32_t *done,
                                                            int32_t *jlen, int32_t *iters, double tol2, double *hn_out) {
    const int s = blockIdx.x;
    if (done[s]) return;
    const double hn = sqrt(sum_items(partial, n_items, 0, item_off[s], item_off[s + 1]));
    if (threadIdx.x != 0) return;
    double *Hs = H + (int64_t)s * (m + 1) * m;
    double *c = cs + (int64_t)s * (m + 1), *sv = sn + (int64_t)s * (m + 1), *gs = g + (int64_t)s * (m + 1);
    Hs[(j + 1) * m + j] = hn;
    hn_out[(int64_t)s * (m + 1)] = hn;
    for (int i = 0; i < j; ++i) {
        const double a = Hs[i * m + j], b = Hs[(i + 1) * m + j];
        Hs[i * m + j] = c[i] * a + sv[i] * b;
        Hs[(i + 1) * m + j] = -sv[i] * a + c[i] * b;
    }
    const double a = Hs[j * m + j], b = Hs[(j + 1) * m + j];
    const double den = sqrt(a * a + b * b);
    c[j] = den > 0.0 ? a / den : 1.0;
    sv[j] = den > 0.0 ? b / den : 0.0;
    Hs[j * m + j] = den;
    Hs[(j + 1) * m + j] = 0.0;
    gs[j + 1] = -sv[j] * gs[j];
    gs[j] = c[j] * gs[j];
    jlen[s] = j + 1;
    iters[s] += 1;
    const double est = gs[j + 1] * gs[j + 1];
    SC(S_RR) = est;
    if (est <= tol2 * SC(S_BB) || hn == 0.0) done[s] = 1;
}

// y = H^{-1} g on the jlen x jlen upper triangle, per system
__global__ void k_gm_solve(int32_t nsys, int m, const double *H, const double *g, const int32_t *jlen, double *y) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsys) return;
    const int j = jlen[s];
    const double *Hs = H + (int64_t)s * (m + 1) * m;
    const double *gs = g + (int64_t)s * (m + 1);
    double *ys = y + (int64_t)s * (m + 1);
    for (int i = m; i >= 0; --i) ys[i] = 0.0;
    for (int i = j - 1; i >= 0; --i) {
        double acc = gs[i];
        for (int k = i + 1; k < j; ++k) acc -= Hs[i * m + k] * ys[k];
        const double d = Hs[i * m + i];
        ys[i] = d != 0.0 ? acc / d : 0.0;
    }
}

// x += sum_i y_i Z_i (all systems; y = 0 beyond jlen)
__global__ __launch_bounds__(kVecThreads) void k_gm_update(const Item *__restrict__ items, int m, int jmax, int64_t ld,
                                                           const double *__restrict__ Z, const double *__restrict__ y,
                                                           const int32_t *__restrict__ jlen, double *x) {
    const Item it = items[blockIdx.x];
    const double *ys = y + (int64_t)it.sys * (m + 1);
    const int js = min(jmax, jlen[it.sys]);      // columns this system built in the cycle
    for (int64_t e = it.beg + threadIdx.x; e < it.end; e += kVecThreads) {
        double acc = x[e];
        for (int i = 0; i < js; ++i) acc += ys[i] * Z[i * ld + e];
        x[e] = acc;
    }
}

#undef SC

// ------------------------------------------------------------------ helpers
inline const int32_t *done_none(cbs_system *h) { return h->flags.get() + h->n_sys; }   // all-zero mask

void dots(cbs_system *h, int K, const double *a0, const double *b0, const double *a1 = nullptr,
          const double *b1 = nullptr, const double *a2 = nullptr, const double *b2 = nullptr,
          const int32_t *mask = nullptr) {
    hipLaunchKernelGGL(k_dots, dim3(h->n_items), dim3(kVecThreads), 0, h->stream, h->items.get(), h->n_items,
                       mask ? mask : h->done.get(), K, a0, b0, a1, b1, a2, b2, h->partial.get());
    LAUNCHCHK();
}

void fin(cbs_system *h, int phase, double tol2, const int32_t *restart_mask = nullptr) {
    hipLaunchKernelGGL(k_fin, dim3(h->n_sys), dim3(kFinThreads), 0, h->stream, phase, h->n_sys, h->item_off.get(),
                       h->n_items, h->partial.get(), h->scal.get(), h->done.get(), h->flags.get(),
                       h->done.get() + 2 * h->n_sys, tol2, restart_mask);
    LAUNCHCHK();
}

int32_t *iters_ptr(cbs_system *h) { return h->done.get() + 2 * h->n_sys; }

// ------------------------------------------------------------------ V-cycle
template <typename T> T *vptr(DArr<char> &a) { return reinterpret_cast<T *>(a.get()); }

template <typename T>
const T *level_vals(Level &L, bool tr);
template <>
const double *level_vals<double>(Level &L, bool tr) { return tr ? L.sell.v64T.get() : L.sell.v64.get(); }
template <>
const float *level_vals<float>(Level &L, bool tr) { return tr ? L.sell.v32T.get() : L.sell.v32.get(); }

template <typename T>
const T *ilu_vals(Level &L, bool tr);
template <>
const double *ilu_vals<double>(Level &L, bool tr) { return tr ? L.iluS64T.get() : L.iluS64.get(); }
template <>
const float *ilu_vals<float>(Level &L, bool tr) { return tr ? L.iluS32T.get() : L.iluS32.get(); }

// One DILU or block ILU(0) smoothing step x <- x + M^{-1}(b - A x)
// (zero_guess: x <- M^{-1} b).  Both have M = (E + L) E^{-1} (E + U): DILU
// with A's own off-diagonal blocks, ILU(0) with those of its factor.
template <typename T>
void dilu_smooth(cbs_system *h, Level &L, bool tr, const T *b, T *x, bool zero_guess) {
    const T *val = level_vals<T>(L, tr);
    const T *fv = L.ilu ? ilu_vals<T>(L, tr) : nullptr;
    const double *Einv = tr ? L.EinvT.get() : L.Einv.get();
    T *y = vptr<T>(L.vt);
    const int ncol = (int)L.colour_off.size() - 1;
    const SellView S = L.sell.view(sizeof(T) == 4);
    auto cnt = [&](int c) { return L.colour_off[c + 1] - L.colour_off[c]; };
    // with two colours the kernels know every neighbour's colour without
    // reading it: the other one
    const int32_t *colour = ncol <= 2 ? nullptr : L.colour.get();
    for (int c = 0; c < ncol; ++c)
        launch_dilu_fwd<T>(h->n, S, val, fv, colour, c, L.sell.cpos[c], cnt(c), Einv, b, x, y, zero_guess,
                           c == ncol - 1, h->stream);
    // the last colour's backward step changes nothing; its forward launch
    // already made its update
    for (int c = ncol - 2; c >= 0; --c)
        launch_dilu_bwd<T>(h->n, S, fv ? fv : val, colour, c, L.sell.cpos[c], cnt(c), Einv, y, x, zero_guess,
                           h->stream);
}

// One symmetric block Gauss-Seidel step in place: the colour classes in
// order, then in reverse (the oracle's order: colour first, then row).  The
// last colour's second pass is left out: nothing it reads changed since its
// first, so it would recompute the same values.
template <typename T>
void sgs_smooth(cbs_system *h, Level &L, bool tr, const T *b, T *x) {
    const T *val = level_vals<T>(L, tr);
    const double *Dinv = tr ? L.DinvT.get() : L.Dinv.get();
    const int ncol = (int)L.colour_off.size() - 1;
    const SellView S = L.sell.view(sizeof(T) == 4);
    auto colour = [&](int c) {
        launch_gs_colour<T>(h->n, S, val, L.sell.cpos[c], L.colour_off[c + 1] - L.colour_off[c], Dinv, b, x,
                            h->stream);
    };
    for (int c = 0; c < ncol; ++c) colour(c);
    for (int c = ncol - 2; c >= 0; --c) colour(c);
}

// Levels whose colouring has two classes (hex meshes are bipartite).  Colour
// 0 has no earlier neighbours, so its DILU / ILU(0) pivot is its diagonal
// block, and with two colours the ILU(0) factor keeps A's off-diagonal
// blocks.  One DILU or ILU(0) step from x, y_0 = E_0^{-1} r_0, y_1 = E_1^{-1}
// (r_1 - A_10 y_0), z_0 = y_0 - E_0^{-1} A_01 y_1, is then the same as
//   x_0 = E_0^{-1} (b_0 - A_01 x_1);  x_1 += E_1^{-1} (b_1 - A_1. x);
//   x_0 = E_0^{-1} (b_0 - A_01 x_1)
// and a symmetric Gauss-Seidel step is the same with D for E and the
// replacement x_1 = D_1^{-1} (b_1 - A_10 x_0).  Both give the same update up
// to rounding order.  A step's first colour-0 update repeats the last one of
// the step before (x_1 has not changed since), so `steps` steps take one
// colour-0 launch more than colour-1 launches.  After them the residual of
// colour 0 is zero; rz, when given, gets those zeros.
template <typename T>
void smooth_two_colour(cbs_system *h, Level &L, bool tr, const T *b, T *x, int steps, bool zero_guess, T *rz) {
    if (steps <= 0) return;
    const T *val = level_vals<T>(L, tr);
    const double *P = L.dilu ? (tr ? L.EinvT.get() : L.Einv.get()) : (tr ? L.DinvT.get() : L.Dinv.get());
    const SellView S = L.sell.view(sizeof(T) == 4);
    const int32_t n0 = L.colour_off[1] - L.colour_off[0], n1 = L.colour_off[2] - L.colour_off[1];
    auto c0 = [&](int form, T *z) { launch_gs_colour<T>(h->n, S, val, L.sell.cpos[0], n0, P, b, x, h->stream, form, z); };
    auto c1 = [&](int form) { launch_gs_colour<T>(h->n, S, val, L.sell.cpos[1], n1, P, b, x, h->stream, form); };
    c0(zero_guess ? 2 : 0, nullptr);                 // from zero: every x_1 is still zero
    for (int s = 0; s < steps; ++s) {
        // DILU's colour-1 update is a correction of x_1, except from zero
        c1(L.dilu && !(zero_guess && s == 0) ? 1 : 0);
        c0(0, s == steps - 1 ? rz : nullptr);
    }
}

// the positions [p0, p1) of a colour-ordered copy as a copy of their own
// (p0 a whole number of slices)
SellView position_range(SellView S, int32_t p0, int32_t p1) {
    if (p0 & ((1 << S.lc) - 1)) cbs_throw(CBS_ERR_ARG, "colour range not slice-aligned");
    const int32_t s0 = p0 >> S.lc;
    S.N = p1 - p0;
    S.soff += s0;
    S.sw += s0;
    S.prow += p0;
    return S;
}

// x = V(b) with zero initial guess on level l; the result lands in x.  When
// rfine is given, b is not yet formed: it is the restriction of the finer
// level's residual rfine, which the first kernel of this level computes and
// stores into b (fused into the zero-guess sweep when there is one).  On
// level 0 of a mixed-precision cycle, b64 is the FP64 right side (rounded
// into b by the first kernel) and the result goes widened to x64 instead.
//
// zero = false (levels below the finest only, rfine null): x holds a start
// and b the level's right side, both left by an earlier cycle on this level,
// whose zero-guess sweep also left c = D^{-1} b behind.  This is the second
// run of a W-cycle's coarse correction.
template <typename T>
void vcycle(cbs_system *h, bool tr, int l, T *b, T *x, const T *rfine, const double *b64 = nullptr,
            double *x64 = nullptr, bool zero = true) {
    hipStream_t st = h->stream;
    const cbs_options &o = h->opt;
    const int n = h->n;
    const int nlev = (int)h->lev.size();
    Level &L = h->lev[l];
    const int64_t m = (int64_t)L.N * n;
    const int nu1 = std::max(0, o.pre_sweeps), nu2 = std::max(0, o.post_sweeps);
    const double om = level_omega(o, l);
    constexpr bool fp32 = sizeof(T) == sizeof(float);
    const bool bj = l < nlev - 1 && !L.dilu && !L.sgs;
    const bool fuse_in = fp32 && b64 && bj && nu1 >= 1;
    const bool fuse_out = fp32 && x64 && bj && nu2 >= 1;
    if (b64 && !fuse_in) launch_cast<double, T>(m, b64, b, st);
    auto finish = [&] {
        if (x64 && !fuse_out) launch_cast<T, double>(m, x, x64, st);
    };
    auto restrict_into_b = [&] {
        const Level &F = h->lev[l - 1];
        launch_restrict<T>(n, L.N, F.agg_ptr.get(), F.agg_mem.get(), rfine, b, st);
    };
    if (!zero && (rfine || b64 || l == 0 || l == nlev - 1 || l == tail_level_for(h, sizeof(T))))
        cbs_throw(CBS_ERR_ARG, "V-cycle from a start: not on this level");
    // the coarse correction: the next level's cycle, twice on the w_levels
    // finest levels (the second run from the first one's result), once where
    // the next level is the coarsest (solved exactly)
    auto coarse = [&](T *bc, T *xc, const T *r) {
        vcycle<T>(h, tr, l + 1, bc, xc, r);
        if (l < o.w_levels && l + 2 < nlev) vcycle<T>(h, tr, l + 1, bc, xc, nullptr, nullptr, nullptr, false);
    };
    if (rfine && l == tail_level_for(h, sizeof(T))) {        // the rest of the cycle in one workgroup
        launch_tail<T>(h, tr, l, rfine);
        return;
    }
    if (l == nlev - 1) {
        if (rfine) restrict_into_b();
        launch_coarse_solve(h, tr, b, x, fp32);
        finish();
        return;
    }
    const T *val = level_vals<T>(L, tr);
    const double *Dinv = tr ? L.DinvT.get() : L.Dinv.get();
    T *tmp = vptr<T>(L.vt);
    T *r = vptr<T>(L.vr);
    Level &C = h->lev[l + 1];
    T *bc = vptr<T>(C.vb), *xc = vptr<T>(C.vx);
    if (L.dilu || L.sgs) {
        if (rfine) restrict_into_b();
        const bool two = L.colour_off.size() == 3 && L.sell.cpos.size() == 3;
        if (two && nu1 >= 1) {
            // colour 0's residual is zero after the steps: only colour 1's is formed
            smooth_two_colour<T>(h, L, tr, b, x, nu1, zero, r);
            launch_rows<T, T>(1, n, position_range(L.sell.view(fp32), L.sell.cpos[1], L.sell.cpos[2]), val, x, b, r,
                              nullptr, 0.0, st);
        } else {
            if (zero && (L.sgs || nu1 == 0)) launch_fill<T>(m, x, st);    // Gauss-Seidel starts from x = 0
            for (int s = 0; s < nu1; ++s) {
                if (L.dilu) dilu_smooth<T>(h, L, tr, b, x, zero && s == 0);
                else sgs_smooth<T>(h, L, tr, b, x);
            }
            launch_rows<T, T>(1, n, L.sell.view(fp32), val, x, b, r, nullptr, 0.0, st);
        }
        coarse(bc, xc, r);
        launch_prolong<T>(n, L.N, L.agg.get(), xc, x, st);
        if (two) {
            smooth_two_colour<T>(h, L, tr, b, x, nu2, false, nullptr);
        } else {
            for (int s = 0; s < nu2; ++s) {
                if (L.dilu) dilu_smooth<T>(h, L, tr, b, x, false);
                else sgs_smooth<T>(h, L, tr, b, x);
            }
        }
        finish();
        return;
    }
    const int switches = zero ? (nu1 >= 1 ? nu1 - 1 : 0) + nu2 : nu1 + nu2;
    T *cur = (switches % 2 == 0) ? x : tmp;
    T *oth = (cur == x) ? tmp : x;
    if (!zero && cur != x) launch_cast<T, T>(m, x, cur, st);
    // FP32 sweeps run on the row-scaled values Dinv A (D^{-T} A^T in the
    // transposed solve) against c = Dinv b, which the zero-guess sweep leaves
    // behind
    const bool scaled = fp32 && (tr ? L.scaledT : L.scaled);
    const T *sval = scaled ? reinterpret_cast<const T *>(tr ? L.sod.v32T.get() : L.sod.v32.get()) : nullptr;
    T *c = scaled ? vptr<T>(L.vc) : nullptr;
    // pagg/pe: sweep from x + P e (the prolongation fused into the sweep);
    // y64: write the result widened to FP64 there instead of into `to`
    auto sweep = [&](T *from, T *to, const int32_t *pagg, const T *pe, double *y64) {
        if (scaled)
            launch_rows<T, T>(4, n, L.sod.view(true), sval, from, c, to, nullptr, om, st, nullptr, pagg, pe,
                              y64);
        else
            launch_rows<T, T>(2, n, L.sell.view(fp32), val, from, b, to, Dinv, om, st, nullptr, pagg, pe, y64);
    };
    if (!zero) {
        for (int s = 0; s < nu1; ++s) {
            sweep(cur, oth, nullptr, nullptr, nullptr);
            std::swap(cur, oth);
        }
    } else if (nu1 >= 1) {
        if (fuse_in) {
            if constexpr (fp32)
                launch_cast_sweep0(n, L.N, b64, b, Dinv, om, cur, c, st);
        } else if (rfine) {
            launch_restrict_sweep0<T>(n, L.N, h->lev[l - 1].agg_ptr.get(), h->lev[l - 1].agg_mem.get(), rfine, b,
                                      Dinv, om, cur, c, st);
        } else {
            launch_rows<T, T>(3, n, L.sell.view(fp32), val, cur, b, cur, Dinv, om, st, c);
        }
        for (int s = 1; s < nu1; ++s) {
            sweep(cur, oth, nullptr, nullptr, nullptr);
            std::swap(cur, oth);
        }
    } else {
        if (rfine) restrict_into_b();
        if (scaled && nu2 > 0)   // c only; oth is scratch here
            launch_rows<T, T>(3, n, L.sell.view(true), val, oth, b, oth, Dinv, om, st, c);
        launch_fill<T>(m, cur, st);
    }
    launch_rows<T, T>(1, n, L.sell.view(fp32), val, cur, b, r, Dinv, om, st);
    coarse(bc, xc, r);
    // On large levels the extra aggregate-map gathers cost more than the
    // separate prolongation pass; on small ones the saved launch wins.
    const bool fuse_pro = nu2 > 0 && L.N < kSmallLevelRows;
    if (!fuse_pro) launch_prolong<T>(n, L.N, L.agg.get(), xc, cur, st);
    for (int s = 0; s < nu2; ++s) {
        const bool first = s == 0 && fuse_pro, last = s == nu2 - 1 && fuse_out;
        sweep(cur, oth, first ? L.agg.get() : nullptr, first ? xc : nullptr, last ? x64 : nullptr);
        std::swap(cur, oth);
    }
    finish();
}

}  // namespace

// FP64 operator of the Krylov loop: level 0 in the internal numbering
void spmv64(cbs_system *h, const double *x, double *y, bool transposed) {
    Level &L0 = h->lev[0];
    const double *val = transposed ? L0.sell.v64T.get() : L0.sell.v64.get();
    launch_rows<double, double>(0, h->n, L0.sell.view(), val, x, nullptr, y, nullptr, 0.0, h->stream);
}

static void residual64(cbs_system *h, const double *b, const double *x, double *r, bool transposed) {
    Level &L0 = h->lev[0];
    const double *val = transposed ? L0.sell.v64T.get() : L0.sell.v64.get();
    launch_rows<double, double>(1, h->n, L0.sell.view(), val, x, b, r, nullptr, 0.0, h->stream);
}

void precond_apply(cbs_system *h, const double *r, double *z, bool tr) {
    const int n = h->n;
    const int64_t m = (int64_t)h->N * n;
    hipStream_t st = h->stream;
    switch (h->opt.precond) {
        case CBS_PREC_NONE:
            launch_copy(m, r, z, st);
            return;
        case CBS_PREC_BJACOBI:
            launch_block_apply(n, h->N, tr ? h->lev[0].DinvT.get() : h->lev[0].Dinv.get(), r, z, st);
            return;
        case CBS_PREC_SGS: {
            Level &L0 = h->lev[0];
            const int steps = std::max(1, h->opt.pre_sweeps);
            if (L0.colour_off.size() == 3 && L0.sell.cpos.size() == 3) {
                smooth_two_colour<double>(h, L0, tr, r, z, steps, true, nullptr);
                return;
            }
            launch_fill<double>(m, z, st);
            for (int s = 0; s < steps; ++s) sgs_smooth<double>(h, L0, tr, r, z);
            return;
        }
        default:
            break;
    }
    if (h->opt.precision == CBS_PRECISION_MIXED) {
        Level &L0 = h->lev[0];
        float *b32 = vptr<float>(L0.vb), *x32 = vptr<float>(L0.vx);
        vcycle<float>(h, tr, 0, b32, x32, nullptr, r, z);
    } else {
        vcycle<double>(h, tr, 0, const_cast<double *>(r), z, nullptr);
    }
}

// ------------------------------------------------------------------ drivers
namespace {

struct HostView {
    std::vector<double> scal;
    std::vector<int32_t> state;     // done | flags | iters
};

void read_state(cbs_system *h, HostView &hv, bool with_scal) {
    hipStream_t st = h->stream;
    hv.state.resize(3 * h->n_sys);
    HIPCHK(hipMemcpyAsync(hv.state.data(), h->done.get(), sizeof(int32_t) * 3 * h->n_sys, hipMemcpyDeviceToHost, st));
    if (with_scal) {
        hv.scal.resize(S_NSCAL * h->n_sys);
        HIPCHK(hipMemcpyAsync(hv.scal.data(), h->scal.get(), sizeof(double) * S_NSCAL * h->n_sys,
                              hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
}

// keep the recurrence's ||r||^2 (S_RR) of every system in S_RREC before a
// true residual overwrites it
void save_recursive(cbs_system *h) {
    const int nsys = h->n_sys;
    HIPCHK(hipMemcpyAsync(h->scal.get() + (size_t)S_RREC * nsys, h->scal.get() + (size_t)S_RR * nsys,
                          sizeof(double) * nsys, hipMemcpyDeviceToDevice, h->stream));
}

// true residual r = b - A x of every system -> S_RR
void true_residual(cbs_system *h, const double *b, const double *x, bool tr) {
    residual64(h, b, x, h->r.get(), tr);
    dots(h, 1, h->r.get(), h->r.get(), nullptr, nullptr, nullptr, nullptr, done_none(h));
    fin(h, PH_TRUE, 0.0);
}

// One right-preconditioned BiCGStab iteration for every unfinished system,
// in two halves: the first ends with s = r - alpha v and the half-step test
// on ||s||, the second applies the preconditioner to s and finishes.  Only
// kernel launches on h->stream (no memset/memcpy, no host sync), so each
// part can be captured once and replayed as a graph.
void bicg_half1(cbs_system *h, bool tr) {
    hipStream_t st = h->stream;
    const double tol2 = h->opt.tol * h->opt.tol;
    const int nsys = h->n_sys;
    double *r = h->r.get(), *rh = h->rh.get(), *p = h->p.get(), *v = h->v.get();
    double *ph = h->ph.get(), *sv = h->s.get();
    const Item *items = h->items.get();
    const dim3 G(h->n_items), B(kVecThreads);
    hipLaunchKernelGGL(k_p_update, G, B, 0, st, items, nsys, h->done.get(), h->scal.get(), h->flags.get(), r, p, v);
    precond_apply(h, p, ph, tr);
    spmv64(h, ph, v, tr);
    dots(h, 1, rh, v);
    fin(h, PH_ALPHA, tol2);
    hipLaunchKernelGGL(k_s_update, G, B, 0, st, items, h->n_items, nsys, h->done.get(), h->scal.get(), h->flags.get(),
                       r, v, sv, h->partial.get());
    LAUNCHCHK();
}

// x and r updates and the end-of-iteration scalars
void bicg_finish(cbs_system *h, double *x) {
    hipStream_t st = h->stream;
    const double tol2 = h->opt.tol * h->opt.tol;
    const dim3 G(h->n_items), B(kVecThreads);
    hipLaunchKernelGGL(k_xr_update, G, B, 0, st, h->items.get(), h->n_items, h->n_sys, h->done.get(), h->scal.get(),
                       h->flags.get(), x, h->ph.get(), h->sh.get(), h->r.get(), h->s.get(), h->t.get(), h->rh.get(),
                       h->partial.get());
    fin(h, PH_END, tol2);
    LAUNCHCHK();
}

void bicg_half2(cbs_system *h, double *x, bool tr) {
    const double tol2 = h->opt.tol * h->opt.tol;
    double *sv = h->s.get(), *sh = h->sh.get(), *t = h->t.get();
    precond_apply(h, sv, sh, tr);
    spmv64(h, sh, t, tr);
    dots(h, 2, t, sv, t, t);
    fin(h, PH_OMEGA, tol2);
    bicg_finish(h, x);
}

enum { PART_FULL = 0, PART_HALF1, PART_HALF2 };

// The whole iteration tests ||s|| with omega (the result of a half-step
// convergence is then exact, only nothing is skipped); the first half alone
// ends with the test so that the host can skip the second.
void bicg_part(cbs_system *h, double *x, bool tr, int part) {
    if (part != PART_HALF2) bicg_half1(h, tr);
    if (part == PART_HALF1) fin(h, PH_SNORM, h->opt.tol * h->opt.tol);
    if (part != PART_HALF1) bicg_half2(h, x, tr);
}

// Replay a captured part of the iteration (captured on first use).
void bicg_part_graph(cbs_system *h, double *xw, bool tr, int part) {
    hipGraphExec_t &ex = h->g_iter[part][tr ? 1 : 0];
    if (!ex) {
        if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
        hipStream_t saved = h->stream;
        h->stream = h->cap_stream;
        hipGraph_t g = nullptr;
        try {
            HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed));
            bicg_part(h, xw, tr, part);
            HIPCHK(hipStreamEndCapture(h->cap_stream, &g));
        } catch (...) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(h->cap_stream, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            h->stream = saved;
            throw;
        }
        h->stream = saved;
        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) { ex = nullptr; cbs_throw(CBS_ERR_HIP, "hipGraphInstantiate failed"); }
    }
    HIPCHK(hipGraphLaunch(ex, h->stream));
}

int bicgstab(cbs_system *h, const double *b, double *x, bool tr, std::vector<int> &status) {
    hipStream_t st = h->stream;
    const cbs_options &o = h->opt;
    const double tol2 = o.tol * o.tol;
    const int nsys = h->n_sys;
    double *r = h->r.get(), *rh = h->rh.get(), *p = h->p.get(), *v = h->v.get();
    double *ph = h->ph.get(), *sv = h->s.get(), *sh = h->sh.get(), *t = h->t.get();
    const Item *items = h->items.get();
    const dim3 G(h->n_items), B(kVecThreads);
    int32_t *rmask = h->flags.get() + 2 * nsys;     // restart mask scratch
    (void)sv; (void)sh; (void)t; (void)ph;

    residual64(h, b, x, r, tr);
    dots(h, 2, r, r, b, b, nullptr, nullptr, done_none(h));
    fin(h, PH_INIT, tol2);
    hipLaunchKernelGGL(k_zero_if_bzero, G, B, 0, st, items, nsys, h->scal.get(), x);
    HIPCHK(hipMemcpyAsync(rh, r, sizeof(double) * (size_t)h->N * h->n, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemsetAsync(p, 0, sizeof(double) * (size_t)h->N * h->n, st));
    HIPCHK(hipMemsetAsync(v, 0, sizeof(double) * (size_t)h->N * h->n, st));

    std::vector<int> bd_restarts(nsys, 0), tr_restarts(nsys, 0);
    status.assign(nsys, CBS_NOT_CONVERGED);
    HostView hv;
    int it = 0;
    const int every = std::max(1, o.check_every);
    const bool graphs = x == h->xw.get();
    bool split = false;          // next iteration in two halves with a check between
    for (;;) {
        bool check = (it % every == 0) || it >= o.max_iter;
        if (check) {
            read_state(h, hv, false);
            const int32_t *dn = hv.state.data(), *fl = dn + nsys;
            bool all_done = true, any_bd = false;
            for (int s = 0; s < nsys; ++s) {
                if (status[s] == CBS_ERR_BREAKDOWN) continue;
                if (!dn[s]) all_done = false;
                if (fl[s] & 1) any_bd = true;
            }
            if (any_bd) {
                // restart broken systems once from the true residual
                std::vector<int32_t> mask(nsys, 0);
                for (int s = 0; s < nsys; ++s) {
                    if (status[s] == CBS_ERR_BREAKDOWN || !(fl[s] & 1)) continue;
                    if (bd_restarts[s]++ >= 1) { status[s] = CBS_ERR_BREAKDOWN; mask[s] = 0; }
                    else mask[s] = 1;
                }
                HIPCHK(hipMemcpyAsync(rmask, mask.data(), sizeof(int32_t) * nsys, hipMemcpyHostToDevice, st));
                residual64(h, b, x, h->w.get(), tr);
                hipLaunchKernelGGL(k_mask_copy, G, B, 0, st, items, rmask, 1, h->w.get(), r);
                hipLaunchKernelGGL(k_mask_copy, G, B, 0, st, items, rmask, 1, h->w.get(), rh);
                hipLaunchKernelGGL(k_mask_copy, G, B, 0, st, items, rmask, 1, nullptr, p);
                hipLaunchKernelGGL(k_mask_copy, G, B, 0, st, items, rmask, 1, nullptr, v);
                dots(h, 1, r, r, nullptr, nullptr, nullptr, nullptr, done_none(h));
                fin(h, PH_RESTART, tol2, rmask);
                // systems out of restarts stay frozen: mark them done
                for (int s = 0; s < nsys; ++s)
                    if (status[s] == CBS_ERR_BREAKDOWN) {
                        int32_t one = 1;
                        HIPCHK(hipMemcpyAsync(h->done.get() + s, &one, sizeof(int32_t), hipMemcpyHostToDevice, st));
                        HIPCHK(hipStreamSynchronize(st));
                    }
                continue;
            }
            if (all_done) {
                // verify with the true residual; restart systems that fall short
                save_recursive(h);
                true_residual(h, b, x, tr);
                read_state(h, hv, true);
                std::vector<int32_t> mask(nsys, 0);
                bool any = false;
                for (int s = 0; s < nsys; ++s) {
                    if (status[s] == CBS_ERR_BREAKDOWN) continue;
                    const double bb = hv.scal[S_BB * nsys + s], rr = hv.scal[S_RR * nsys + s];
                    if (bb == 0.0 || rr <= tol2 * bb) status[s] = CBS_OK;
                    else if (it < o.max_iter && tr_restarts[s]++ < 50) { mask[s] = 1; any = true; }
                }
                if (!any) break;
                HIPCHK(hipMemcpyAsync(rmask, mask.data(), sizeof(int32_t) * nsys, hipMemcpyHostToDevice, st));
                hipLaunchKernelGGL(k_mask_copy, G, B, 0, st, items, rmask, 1, r, rh);
                hipLaunchKernelGGL(k_mask_copy, G, B, 0, st, items, rmask, 1, nullptr, p);
                hipLaunchKernelGGL(k_mask_copy, G, B, 0, st, items, rmask, 1, nullptr, v);
                dots(h, 1, r, r, nullptr, nullptr, nullptr, nullptr, done_none(h));
                fin(h, PH_RESTART, tol2, rmask);
                continue;
            }
        }
        if (it >= o.max_iter) { save_recursive(h); break; }
        if (check) {
            // Near convergence (every unfinished system flagged by the end of
            // the last iteration) run the iteration in halves: if every
            // unfinished system already meets the tolerance with s, the second
            // preconditioner application and product are skipped.
            const int32_t *dn = hv.state.data(), *fl = dn + nsys;
            split = true;
            for (int s = 0; s < nsys && split; ++s)
                if (!dn[s] && !(fl[s] & kFlagBreak) && !(fl[s] & kFlagNear)) split = false;
        }
        if (!split) {
            if (graphs) bicg_part_graph(h, x, tr, PART_FULL);
            else bicg_part(h, x, tr, PART_FULL);
        } else {
            if (graphs) bicg_part_graph(h, x, tr, PART_HALF1);
            else bicg_part(h, x, tr, PART_HALF1);
            read_state(h, hv, false);
            const int32_t *dn = hv.state.data(), *fl = dn + nsys;
            bool all_half = true;
            for (int s = 0; s < nsys && all_half; ++s)
                if (!dn[s] && !(fl[s] & kFlagBreak) && !(fl[s] & kFlagHalf)) all_half = false;
            if (all_half) bicg_finish(h, x);
            else if (graphs) bicg_part_graph(h, x, tr, PART_HALF2);
            else bicg_part(h, x, tr, PART_HALF2);
        }
        ++it;
    }
    return it;
}

// Flexible GMRES(m) (Z_j = M^{-1} V_j kept, x += Z y), or with flexible ==
// false right-preconditioned GMRES(m): only V is kept, the preconditioned
// vector is formed for the product and dropped, and each cycle ends with
// x += M^{-1} (V y) -- one more preconditioner application per cycle and m
// fewer stored vectors.
int fgmres(cbs_system *h, const double *b, double *x, bool tr, std::vector<int> &status) {
    hipStream_t st = h->stream;
    const cbs_options &o = h->opt;
    const bool flexible = o.solver == CBS_SOLVER_FGMRES;
    const double tol2 = o.tol * o.tol;
    const int nsys = h->n_sys;
    const int m = std::max(1, o.restart);
    const int64_t ld = (int64_t)h->N * h->n;
    double *r = h->r.get(), *w = h->w.get();
    double *V = h->V.get(), *Z = h->Z.get();
    const Item *items = h->items.get();
    const dim3 G(h->n_items), B(kVecThreads), GS(nsys), BS(kFinThreads), GS1(cdiv(nsys, 64)), BS1(64);
    double *coef = h->yv.get() + (int64_t)nsys * (m + 1);       // (m+1) per system
    double *hn = coef + (int64_t)nsys * (m + 1);                // 1 per system (stride m+1)
    status.assign(nsys, CBS_NOT_CONVERGED);
    HostView hv;
    int it = 0;
    bool first = true;
    const int every = std::max(1, o.check_every);
    int32_t *iters = iters_ptr(h);
    HIPCHK(hipMemsetAsync(iters, 0, sizeof(int32_t) * nsys, st));
    for (;;) {
        // the least-squares residual of the last cycle (the first cycle: the
        // initial true residual, saved below) before the restart replaces it
        if (!first) save_recursive(h);
        residual64(h, b, x, r, tr);
        dots(h, 2, r, r, b, b, nullptr, nullptr, done_none(h));
        hipLaunchKernelGGL(k_gm_start, GS, BS, 0, st, nsys, m, h->item_off.get(), h->n_items, h->partial.get(),
                           h->scal.get(), h->gvec.get(), h->done.get(), h->flags.get() + 3 * nsys, tol2, first ? 1 : 0);
        if (first) {
            hipLaunchKernelGGL(k_zero_if_bzero, G, B, 0, st, items, nsys, h->scal.get(), x);
            save_recursive(h);
        }
        first = false;
        read_state(h, hv, false);
        bool all_done = true;
        for (int s = 0; s < nsys; ++s) {
            if (hv.state[s]) status[s] = CBS_OK; else all_done = false;
        }
        if (all_done || it >= o.max_iter) break;
        hipLaunchKernelGGL(k_scale, G, B, 0, st, items, h->done.get(), h->scal.get() + S_RHO * nsys, 1, r, V);
        int j = 0;
        for (; j < m && it < o.max_iter; ++j) {
            double *vj = V + j * ld, *zj = flexible ? Z + j * ld : h->ph.get();
            precond_apply(h, vj, zj, tr);
            spmv64(h, zj, w, tr);
            // classical Gram-Schmidt; a second pass re-orthogonalises the
            // systems whose w lost more than 90% of its norm in the first
            int32_t *skip = h->flags.get() + 4 * nsys;
            for (int pass = 0; pass < 2; ++pass) {
                const int32_t *mask = pass == 0 ? h->done.get() : skip;
                hipLaunchKernelGGL(k_mdot, G, B, 0, st, items, h->n_items, mask, j, ld, V, w, h->partial.get(),
                                   pass == 0 ? 1 : 0);
                hipLaunchKernelGGL(k_mdot_fin, GS, BS, 0, st, j, m, h->item_off.get(), h->n_items,
                                   h->partial.get(), mask, h->H.get(), coef, pass, pass == 0 ? skip : nullptr);
                hipLaunchKernelGGL(k_maxpy, G, B, 0, st, items, mask, j, m, ld, V, coef, w);
            }
            dots(h, 1, w, w);
            hipLaunchKernelGGL(k_gm_givens, GS, BS, 0, st, nsys, j, m, h->item_off.get(), h->n_items,
                               h->partial.get(), h->scal.get(), h->H.get(), h->cs.get(), h->sn.get(), h->gvec.get(),
                               h->done.get(), h->flags.get() + 3 * nsys, iters, tol2, hn);
            hipLaunchKernelGGL(k_scale, G, B, 0, st, items, h->done.get(), hn, m + 1, w, V + (j + 1) * ld);
            LAUNCHCHK();
            ++it;
            if ((it % every) == 0) {
                read_state(h, hv, false);
                bool ad = true;
                for (int s = 0; s < nsys; ++s) ad = ad && hv.state[s];
                if (ad) { ++j; break; }
            }
        }
        const int jmax = std::min(j, m);
        hipLaunchKernelGGL(k_gm_solve, GS1, BS1, 0, st, nsys, m, h->H.get(), h->gvec.get(), h->flags.get() + 3 * nsys,
                           h->yv.get());
        if (flexible) {
            hipLaunchKernelGGL(k_gm_update, G, B, 0, st, items, m, jmax, ld, Z, h->yv.get(), h->flags.get() + 3 * nsys,
                               x);
        } else {
            double *u = h->sh.get(), *z = h->ph.get();
            launch_fill<double>(ld, u, st);
            hipLaunchKernelGGL(k_gm_update, G, B, 0, st, items, m, jmax, ld, V, h->yv.get(), h->flags.get() + 3 * nsys,
                               u);
            precond_apply(h, u, z, tr);
            hipLaunchKernelGGL(k_gm_add, G, B, 0, st, items, z, x);
        }
        LAUNCHCHK();
        // next cycle re-evaluates every system from its true residual
        HIPCHK(hipMemsetAsync(h->done.get(), 0, sizeof(int32_t) * nsys, st));
    }
    // final true residual for the statistics
    true_residual(h, b, x, tr);
    return it;
}

}  // namespace

void invalidate_graphs(cbs_system *h) {
    for (auto &part : h->g_iter)
        for (auto &g : part)
            if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
}

void alloc_krylov(cbs_system *h) {
    // any reallocation below would leave the captured graphs pointing at freed buffers
    const void *before[4] = {h->r.get(), h->partial.get(), h->V.get(), h->yv.get()};
    struct Check {
        cbs_system *h;
        const void *const *b;
        ~Check() {
            const void *after[4] = {h->r.get(), h->partial.get(), h->V.get(), h->yv.get()};
            for (int i = 0; i < 4; ++i)
                if (after[i] != b[i]) { invalidate_graphs(h); break; }
        }
    } check{h, before};
    const int64_t m = (int64_t)h->N * h->n;
    const int nsys = h->n_sys;
    for (DArr<double> *a : {&h->r, &h->rh, &h->p, &h->v, &h->ph, &h->s, &h->sh, &h->t, &h->w}) a->ensure(m);
    if (h->opt.solver != CBS_SOLVER_BICGSTAB) {
        const int mr = std::max(1, h->opt.restart);
        h->V.ensure((size_t)(mr + 1) * m);
        if (h->opt.solver == CBS_SOLVER_FGMRES) h->Z.ensure((size_t)mr * m);
        h->H.ensure((size_t)nsys * (mr + 1) * mr);
        h->gvec.ensure((size_t)nsys * (mr + 1));
        h->cs.ensure((size_t)nsys * (mr + 1));
        h->sn.ensure((size_t)nsys * (mr + 1));
        h->yv.ensure((size_t)nsys * (mr + 1) * 3);
    }
    const int K = std::max(3, h->opt.solver != CBS_SOLVER_BICGSTAB ? h->opt.restart + 2 : 3);
    h->partial.ensure((size_t)K * h->n_items);
}

int krylov_solve(cbs_system *h, const double *b, double *x, cbs_stats *stv, bool tr) {
    hipStream_t st = h->stream;
    const int nsys = h->n_sys;
    if (tr) amg_build_transposed(h);
    check_finite(b, (int64_t)h->N * h->n, h->dflag.get(), st);
    alloc_krylov(h);
    HIPCHK(hipMemsetAsync(h->flags.get(), 0, sizeof(int32_t) * 5 * nsys, st));
    HIPCHK(hipMemsetAsync(h->done.get(), 0, sizeof(int32_t) * 3 * nsys, st));
    HIPCHK(hipEventRecord(h->ev0, st));
    std::vector<int> status;
    // the solvers run on work copies in the internal numbering (the captured
    // iteration graph points at xw)
    const int64_t m = (int64_t)h->N * h->n;
    h->xw.ensure(m);
    h->bw.ensure(m);
    const double *bi = b;
    if (h->renumbered) {
        permute_vec(h, b, h->bw.get(), true);
        permute_vec(h, x, h->xw.get(), true);
        bi = h->bw.get();
    } else {
        launch_copy(m, x, h->xw.get(), st);
    }
    if (h->opt.solver != CBS_SOLVER_BICGSTAB) fgmres(h, bi, h->xw.get(), tr, status);
    else bicgstab(h, bi, h->xw.get(), tr, status);
    if (h->renumbered) permute_vec(h, h->xw.get(), x, false);
    else launch_copy(m, h->xw.get(), x, st);
    HIPCHK(hipEventRecord(h->ev1, st));
    // statistics: true residual per system (BiCGStab's last step may not have computed it)
    std::vector<double> rr_rec(nsys), res0(nsys), bbv(nsys);
    {
        HostView hv;
        read_state(h, hv, true);
        for (int s = 0; s < nsys; ++s) {
            rr_rec[s] = hv.scal[S_RREC * nsys + s];
            res0[s] = hv.scal[S_RES0 * nsys + s];
            bbv[s] = hv.scal[S_BB * nsys + s];
        }
    }
    true_residual(h, bi, h->xw.get(), tr);
    HostView hv;
    read_state(h, hv, true);
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    int worst = CBS_OK;
    const double tol2 = h->opt.tol * h->opt.tol;
    for (int s = 0; s < nsys; ++s) {
        const double bb = bbv[s], rr = hv.scal[S_RR * nsys + s];
        int stt = status[s];
        if (stt != CBS_ERR_BREAKDOWN) stt = (bb == 0.0 || rr <= tol2 * bb) ? CBS_OK : CBS_NOT_CONVERGED;
        if (stt < 0) worst = std::min(worst, stt);
        else if (worst >= 0) worst = std::max(worst, stt);
        if (stv) {
            cbs_stats &S = stv[s];
            S.iterations = hv.state[2 * nsys + s];
            S.status = stt;
            S.levels = (int32_t)h->lev.size();
            S.precision_fallback = 0;
            S.rel_res_true = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
            S.rel_res_recursive = bb > 0.0 ? std::sqrt(std::max(rr_rec[s], 0.0) / bb) : 0.0;
            S.rel_res_initial = res0[s];
            S.t_convert_ms = h->t_convert_ms;
            S.t_setup_ms = h->t_setup_ms;
            S.t_solve_ms = ms;
            S.op_complexity = h->op_complexity;
        }
    }
    return worst;
}
