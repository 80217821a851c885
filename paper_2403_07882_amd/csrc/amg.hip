// amg.hip -- aggregation-AMG setup on the device.
//
// The paper's GPU solver is aggregation AMG for block-coupled systems whose
// parallel setup rests on graph matching (Sec. 2.3).  Here, per level:
//   1. FP64 block-diagonal inverses D_i^{-1} (Gauss-Jordan, partial pivoting),
//   2. strength weights w_ij = 1/2 (|A_ij|_F + |A_ji|_F) / max(|A_ii|_F, |A_jj|_F),
//   3. handshake matching: every unmatched node proposes to its strongest
//      unmatched neighbour (ties -> smaller index); mutual proposals pair up;
//      a few rounds, then leftovers join their strongest matched neighbour;
//      `match_passes` passes are composed (pass 2 matches the pair graph
//      whose weights are the scalar Galerkin sums of pass 1),
//   4. Galerkin coarse operator A_c(I,J) = sum_{i in I, j in J} A(i,j)
//      (P^T A P with piecewise-constant P), one wavefront per coarse row,
//      duplicates merged in LDS, sums in a fixed order (deterministic),
//   5. coarsest level: dense FP64 inverse of each system's matrix.
// Integer atomics appear only in counting; every order they could perturb is
// re-sorted, so the hierarchy is reproducible run to run.
#include "cbs_internal.h"

#include <algorithm>
#include <cmath>

void build_row_sys(cbs_system *h, Level &L0);

namespace {

// wavefronts per workgroup of the Galerkin kernel: each takes a coarse row
// of its own, and one per workgroup keeps the workgroup barriers from
// making each wait for the slowest row (4 per workgroup was 10-20% slower)
constexpr int kRapWaves = 1;
constexpr int kRapCap = 4096;     // largest candidate list a coarse row may gather
// Coarse rows with at most kRapSmall candidates (pairwise aggregates of short
// rows) take a thread each instead of a wavefront: kRapSmallTpb threads per
// workgroup, each with a sorted list of kRapSmall slots in LDS.
constexpr int kRapSmall = 48;
constexpr int kRapSmallCount = 64;   // the counting pass keeps no values: longer lists fit
constexpr int32_t kRapSmallRows = 16384;
constexpr int kRapSmallTpb = 64;
// slots per thread of the first launch, counting pass and fill pass (the
// fill keeps a sum beside each column: 12 bytes a slot against 4)
constexpr int kRapCountSlots = 32;
constexpr int kRapSlots = 24;
constexpr int kRapListGroups = 1024;   // workgroups of a launch over queued rows
constexpr int kMatchRounds = 4;

// ------------------------------------------------------------------ block inverse
template <int n>
__device__ inline bool gj_inverse(double (&a)[n][2 * n]) {
#pragma unroll
    for (int k = 0; k < n; ++k) {
        int p = k;
        double pv = fabs(a[k][k]);
#pragma unroll
        for (int r = k + 1; r < n; ++r)
            if (fabs(a[r][k]) > pv) { pv = fabs(a[r][k]); p = r; }
        if (!(pv > 0.0) || !isfinite(pv)) return false;
        // swap rows k and p with compile-time row indices only (selects), so
        // the array stays in registers
#pragma unroll
        for (int r = k + 1; r < n; ++r) {
            const bool sw = r == p;
#pragma unroll
            for (int c = 0; c < 2 * n; ++c) {
                const double t = a[k][c];
                a[k][c] = sw ? a[r][c] : t;
                a[r][c] = sw ? t : a[r][c];
            }
        }
        const double piv = a[k][k];
#pragma unroll
        for (int c = 0; c < 2 * n; ++c) a[k][c] /= piv;
#pragma unroll
        for (int r = 0; r < n; ++r) {
            if (r == k) continue;
            const double m = a[r][k];
#pragma unroll
            for (int c = 0; c < 2 * n; ++c) a[r][c] -= m * a[k][c];
        }
    }
    return true;
}

// One thread inverts one block; the workgroup's blocks pass through LDS,
// so both the gather of the diagonal blocks (n*n contiguous values each) and
// the store of the inverses (one contiguous run) are read and written by
// consecutive lanes.
constexpr int kInvThreads = 128;
template <int n>
__global__ __launch_bounds__(kInvThreads) void k_blockinv(int32_t N, const int32_t *__restrict__ dslot,
                                                          const double *__restrict__ val, double *__restrict__ Dinv,
                                                          int32_t *bad) {
    constexpr int nn = n * n;
    __shared__ double sh[kInvThreads * nn];
    __shared__ int32_t ss[kInvThreads];
    const int32_t i0 = blockIdx.x * kInvThreads;
    const int cnt = min(kInvThreads, N - i0);
    const int t = threadIdx.x;
    if (t < cnt) ss[t] = dslot[i0 + t];
    __syncthreads();
    for (int e = t; e < cnt * nn; e += kInvThreads) {
        const int q = e / nn;
        sh[e] = val[(int64_t)ss[q] * nn + (e - q * nn)];
    }
    __syncthreads();
    if (t < cnt) {
        double a[n][2 * n];
#pragma unroll
        for (int r = 0; r < n; ++r)
#pragma unroll
            for (int c = 0; c < 2 * n; ++c) a[r][c] = c < n ? sh[t * nn + r * n + c] : (c - n == r ? 1.0 : 0.0);
        const bool ok = gj_inverse<n>(a);
        if (!ok) atomicMin(bad, i0 + t);
#pragma unroll
        for (int r = 0; r < n; ++r)
#pragma unroll
            for (int c = 0; c < n; ++c) sh[t * nn + r * n + c] = ok ? a[r][n + c] : 0.0;
    }
    __syncthreads();
    double *out = Dinv + (int64_t)i0 * nn;
    for (int e = t; e < cnt * nn; e += kInvThreads) out[e] = sh[e];
}

// per-block transpose: out[k] = in[src_k]^T, src_k = mirror[k] (or k)
template <int n>
__global__ void k_block_transpose(int64_t nb, const int32_t *__restrict__ mirror, const double *__restrict__ in,
                                  double *__restrict__ out) {
    constexpr int nn = n * n;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nb * nn) return;
    const int64_t k = g / nn;
    const int e = (int)(g - k * nn), r = e / n, c = e - r * n;
    const int64_t s = mirror ? (int64_t)mirror[k] : k;
    out[g] = in[s * nn + c * n + r];
}

// ------------------------------------------------------------------ strength
// Frobenius norm of every block, read once (one thread per block; the
// squares are summed in element order)
template <int n>
__global__ void k_block_frob(int64_t nb, const double *__restrict__ val, double *__restrict__ nrm) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nb) return;
    const double *A = val + k * (n * n);
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < n * n; ++e) s += A[e] * A[e];
    nrm[k] = sqrt(s);
}

// w_ij = (||A_ij||_F + ||A_ji||_F) / 2 / max(||A_ii||_F, ||A_jj||_F), from
// the block norms (0 on the diagonal).  Rows of up to 8 blocks (face
// neighbours of a hexahedral cell and itself) issue all their gathers before
// using any (a few dependent loads per row instead of a chain per block);
// longer rows take one block at a time.
__global__ void k_strength(int32_t N, const int32_t *rp, const int32_t *col, const int32_t *mirror,
                           const double *nrm, const double *df, double *w) {
    constexpr int MAXL = 8;
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t r0 = rp[i], len = rp[i + 1] - r0;
    if (len <= MAXL) {
        int32_t j[MAXL], m[MAXL];
#pragma unroll
        for (int e = 0; e < MAXL; ++e) {
            j[e] = e < len ? col[r0 + e] : i;
            m[e] = e < len ? mirror[r0 + e] : r0;
        }
        const double di = df[i];
        double dj[MAXL], a[MAXL], b[MAXL];
#pragma unroll
        for (int e = 0; e < MAXL; ++e) {
            dj[e] = e < len ? df[j[e]] : 0.0;
            a[e] = e < len ? nrm[r0 + e] : 0.0;
            b[e] = e < len ? nrm[m[e]] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < MAXL; ++e) {
            if (e < len) {
                const double den = fmax(di, dj[e]);
                w[r0 + e] = j[e] == i ? 0.0 : (den > 0.0 ? 0.5 * (a[e] + b[e]) / den : 0.0);
            }
        }
        return;
    }
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        const int32_t j = col[k];
        if (j == i) { w[k] = 0.0; continue; }
        const double den = fmax(df[i], df[j]);
        w[k] = den > 0.0 ? 0.5 * (nrm[k] + nrm[mirror[k]]) / den : 0.0;
    }
}

// The same weights with L lanes per row (coarse levels, whose rows are too
// long for the unrolled form): each lane takes every L-th block of the row.
template <int L>
__global__ void k_strength_lanes(int32_t N, const int32_t *rp, const int32_t *col, const int32_t *mirror,
                                 const double *nrm, const double *df, double *w) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t i = (int32_t)(t / L), lane = (int32_t)(t - (int64_t)i * L);
    if (i >= N) return;
    const double di = df[i];
    for (int32_t k = rp[i] + lane; k < rp[i + 1]; k += L) {
        const int32_t j = col[k];
        if (j == i) { w[k] = 0.0; continue; }
        const double den = fmax(di, df[j]);
        w[k] = den > 0.0 ? 0.5 * (nrm[k] + nrm[mirror[k]]) / den : 0.0;
    }
}

// lanes per row for a graph of N rows and nnz entries: about one entry each
inline int lanes_for(int64_t N, int64_t nnz) {
    const int64_t avg = N > 0 ? (nnz + N - 1) / N : 1;
    return avg <= 4 ? 4 : avg <= 8 ? 8 : 16;
}

__global__ void k_diag_norm(int32_t N, const int32_t *dslot, const double *nrm, double *df) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) df[i] = nrm[dslot[i]];
}

__global__ void k_zero_diag_w(int32_t N, const int32_t *rp, const int32_t *col, double *w) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
        if (col[k] == i) w[k] = 0.0;
}

// ------------------------------------------------------------------ matching
// partner: -1 unmatched, -2 excluded (frozen system), >= 0 matched partner
__global__ void k_match_init(int32_t N, const int32_t *row_sys, const int32_t *sys_frozen, int32_t *partner) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    partner[i] = sys_frozen[row_sys[i]] ? -2 : -1;
}

// The strongest admissible neighbour of a row: the largest weight, and of
// equal weights the smallest column.  That order is total, so the L lanes of
// a row each take every L-th entry and their picks reduce to the same
// neighbour whatever the order.
template <int L>
__device__ inline void best_reduce(double &bw, int32_t &best) {
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) {
        const double ow = __shfl_xor(bw, o, L);
        const int32_t ob = __shfl_xor(best, o, L);
        if (ob >= 0 && (ow > bw || (ow == bw && ob < best))) { bw = ow; best = ob; }
    }
}

template <int L>
__global__ void k_match_pick(int32_t N, const int32_t *rp, const int32_t *col, const double *w,
                             const int32_t *partner, int32_t *cand) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t i = (int32_t)(t / L), lane = (int32_t)(t - (int64_t)i * L);
    const bool act = i < N;                       // every lane joins the reduction
    int32_t best = -1;
    double bw = 0.0;
    if (act && partner[i] == -1) {
        for (int32_t k = rp[i] + lane; k < rp[i + 1]; k += L) {
            const int32_t j = col[k];
            const double wk = w[k];
            if (j == i || partner[j] != -1 || !(wk > 0.0)) continue;
            if (wk > bw || (wk == bw && j < best)) { bw = wk; best = j; }
        }
    }
    best_reduce<L>(bw, best);
    if (act && lane == 0) cand[i] = best;
}

__global__ void k_match_confirm(int32_t N, const int32_t *cand, int32_t *partner) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t j = cand[i];
    if (j >= 0 && cand[j] == i) partner[i] = j;
}

template <int L>
__global__ void k_match_rep(int32_t N, const int32_t *rp, const int32_t *col, const double *w,
                            const int32_t *partner, int32_t *rep, int32_t *root) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t i = (int32_t)(t / L), lane = (int32_t)(t - (int64_t)i * L);
    const bool act = i < N;
    const int32_t p = act ? partner[i] : -2;
    int32_t best = -1;
    double bw = 0.0;
    if (p == -1) {                                 // unmatched: join the strongest matched neighbour's pair
        for (int32_t k = rp[i] + lane; k < rp[i + 1]; k += L) {
            const int32_t j = col[k];
            const double wk = w[k];
            if (j == i || partner[j] < 0 || !(wk > 0.0)) continue;
            if (wk > bw || (wk == bw && j < best)) { bw = wk; best = j; }
        }
    }
    best_reduce<L>(bw, best);
    if (!act || lane != 0) return;
    int32_t r = i;
    if (p >= 0) r = min(i, p);
    else if (p == -1 && best >= 0) r = min(best, partner[best]);
    rep[i] = r;
    root[i] = (r == i) ? 1 : 0;
}

// newid: the exclusive scan of the root flags (N + 1 entries); its total,
// the aggregate count, goes to *nc
__global__ void k_match_assign(int32_t N, const int32_t *rep, const int32_t *newid, int32_t *agg, int32_t *nc) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    agg[i] = newid[rep[i]];
    if (i == 0) *nc = newid[N];
}

__global__ void k_copy_int(const int32_t *src, int32_t *dst) { *dst = *src; }

__global__ void k_compose(int32_t N, const int32_t *a2, int32_t *agg) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    agg[i] = a2[agg[i]];
}

__global__ void k_inherit_sys(int32_t N, const int32_t *agg, const int32_t *row_sys, int32_t *rs_c) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    rs_c[agg[i]] = row_sys[i];          // every member writes the same value
}

// ------------------------------------------------------------------ members
__global__ void k_fill_int(int32_t *a, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void k_count_members(int32_t N, const int32_t *agg, int32_t *cnt) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) atomicAdd(&cnt[agg[i]], 1);
}

// members per aggregate, and the summed row lengths (over the graph rp) of
// each aggregate's members: its Galerkin candidate count
__global__ void k_count_members_len(int32_t N, const int32_t *agg, const int32_t *rp, int32_t *cnt, int32_t *len) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t a = agg[i];
    atomicAdd(&cnt[a], 1);
    atomicAdd(&len[a], rp[i + 1] - rp[i]);
}

// *mx = max(*mx, v[0..m)) (grid-stride, 256 threads; one atomic per workgroup)
__global__ __launch_bounds__(256) void k_max_into(int64_t m, const int32_t *v, int32_t *mx) {
    __shared__ int32_t sw[4];
    int32_t b = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x)
        b = max(b, v[k]);
    for (int o = 32; o > 0; o >>= 1) b = max(b, __shfl_xor(b, o, 64));
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = b;
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(mx, max(max(sw[0], sw[1]), max(sw[2], sw[3])));
}

__global__ void k_fill_members(int32_t N, const int32_t *agg, int32_t *fill, int32_t *mem) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    mem[atomicAdd(&fill[agg[i]], 1)] = i;
}

__global__ void k_sort_members(int32_t nc, const int32_t *aptr, int32_t *mem) {
    const int32_t I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    const int32_t b = aptr[I], e = aptr[I + 1];
    for (int32_t a = b + 1; a < e; ++a) {
        const int32_t v = mem[a];
        int32_t q = a - 1;
        while (q >= b && mem[q] > v) { mem[q + 1] = mem[q]; --q; }
        mem[q + 1] = v;
    }
}

// ------------------------------------------------------------------ Galerkin RAP
// pass 0: cnt[I] = number of distinct coarse columns of coarse row I
// pass 1: colc / valc of coarse row I at rpc[I] (columns ascending)
// One wavefront per coarse row: the candidate blocks (coarse column J of
// every block of every member row) are gathered into LDS, duplicates are
// marked (top bit of the slot), every candidate learns the rank d of its
// column among the distinct ones, and the n*n sums of each distinct column
// are spread over the lanes (coalesced block reads).  Each sum runs over
// the candidates in gather order: members ascending, then row slots, the
// order of the CPU reference.
// Candidate count of a coarse row: the blocks of all its member rows.
__global__ void k_rap_maxc(int32_t nc, const int32_t *aptr, const int32_t *amem, const int32_t *rp, int32_t *maxc) {
    const int32_t I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    int32_t c = 0;
    for (int32_t m = aptr[I]; m < aptr[I + 1]; ++m) c += rp[amem[m] + 1] - rp[amem[m]];
    atomicMax(maxc, c);
}

// LDS per wavefront: cap entries of column, slot and rank (cap = the
// level's largest candidate count, rounded up), so light levels keep many
// wavefronts resident.
template <int n, int PASS>
__global__ __launch_bounds__(64 * kRapWaves) void k_rap(int32_t nc, int32_t cap, const int32_t *__restrict__ aptr,
                                                        const int32_t *__restrict__ amem,
                                                        const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col,
                                                        const double *__restrict__ val,
                                                        const int32_t *__restrict__ agg, int32_t *cnt,
                                                        const int32_t *__restrict__ rpc, int32_t *colc,
                                                        double *valc, int32_t *flag) {
    constexpr int nn = n * n;
    constexpr uint32_t kFirst = 0x80000000u;
    extern __shared__ int32_t rap_lds[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int32_t *sJw = rap_lds + (size_t)w * 3 * cap;
    uint32_t *sKw = reinterpret_cast<uint32_t *>(sJw + cap);
    int32_t *sDw = sJw + 2 * cap;
    const int32_t I = blockIdx.x * (int32_t)(blockDim.x >> 6) + w;
    const bool active = I < nc;
    // the candidate list: the blocks of the members' rows, member by member.
    // Up to 64 members: one lane per member reads its row's extent, a scan
    // over the lanes gives each member's offset in the list, and every lane
    // then fills list entries of any member (found by binary search over the
    // offsets), so the dependent loads are not repeated per member.
    __shared__ int32_t sMo[kRapWaves][65], sMk[kRapWaves][64];
    int32_t c = 0;
    const int32_t m0 = active ? aptr[I] : 0, nm = active ? aptr[I + 1] - m0 : 0;
    const bool by_lane = nm <= 64;                   // the same for the whole wavefront
    if (by_lane) {
        int32_t kb = 0, len = 0;
        if (lane < nm) {
            const int32_t i = amem[m0 + lane];
            kb = rp[i];
            len = rp[i + 1] - kb;
        }
        int32_t inc = len;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t v = __shfl_up(inc, o, 64);
            if (lane >= o) inc += v;
        }
        c = __shfl(inc, 63, 64);
        if (lane < nm) { sMo[w][lane] = inc - len; sMk[w][lane] = kb; }
        if (lane == 0) sMo[w][nm] = c;
    }
    __syncthreads();
    if (by_lane) {
        const int32_t cl = min(c, cap);
        for (int32_t q = lane; q < cl; q += 64) {
            int32_t lo = 0, hi = nm - 1;             // last member whose offset is <= q
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (sMo[w][mid] <= q) lo = mid;
                else hi = mid - 1;
            }
            const int32_t k = sMk[w][lo] + (q - sMo[w][lo]);
            sJw[q] = agg[col[k]];
            sKw[q] = (uint32_t)k;
        }
    } else {
        for (int32_t m = m0; m < m0 + nm; ++m) {
            const int32_t i = amem[m];
            const int32_t kb = rp[i], len = rp[i + 1] - kb;
            for (int32_t e = lane; e < len; e += 64) {
                const int32_t q = c + e;
                if (q < cap) { sJw[q] = agg[col[kb + e]]; sKw[q] = (uint32_t)(kb + e); }
            }
            c += len;
        }
    }
    if (active && c > cap && lane == 0) atomicOr(flag, 8);
    __syncthreads();
    const int32_t cc = active ? min(c, cap) : 0;
    for (int32_t q = lane; q < cc; q += 64) {
        const int32_t J = sJw[q];
        bool f = true;
        for (int32_t p = 0; p < q; ++p)
            if (sJw[p] == J) { f = false; break; }
        if (f) sKw[q] |= kFirst;
    }
    __syncthreads();
    if (PASS == 0) {
        int32_t d = 0;
        for (int32_t q = lane; q < cc; q += 64) d += (sKw[q] & kFirst) ? 1 : 0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
        if (active && lane == 0) cnt[I] = d;
        return;
    }
    const int32_t base = active ? rpc[I] : 0;
    for (int32_t q = lane; q < cc; q += 64) {
        const int32_t J = sJw[q];
        int32_t d = 0;
        for (int32_t p = 0; p < cc; ++p) d += ((sKw[p] & kFirst) && sJw[p] < J) ? 1 : 0;
        sDw[q] = d;
        if (sKw[q] & kFirst) colc[base + d] = J;
    }
    __syncthreads();
    // Candidates regrouped by output block, candidate order kept within a
    // group: slot of q = (candidates of lower blocks) + (earlier candidates
    // of its own block).  sJw (columns, no longer needed) takes the list.
    for (int32_t q = lane; q < cc; q += 64) {
        const int32_t d = sDw[q];
        int32_t pos = 0;
        for (int32_t p = 0; p < cc; ++p) {
            const int32_t dp = sDw[p];
            pos += (dp < d || (dp == d && p < q)) ? 1 : 0;
        }
        sJw[pos] = q;
    }
    __syncthreads();
    // where each output block's group starts in the list (up to 64 blocks;
    // sMo is free again), else found by binary search per output value
    const int32_t nd = active ? rpc[I + 1] - base : 0;
    const bool starts = nd <= 64;                    // the same for the whole wavefront
    if (starts) {
        for (int32_t q = lane; q < cc; q += 64) {
            const int32_t dq = sDw[sJw[q]];
            if (q == 0 || sDw[sJw[q - 1]] != dq) sMo[w][dq] = q;
        }
        if (lane == 0) sMo[w][nd] = cc;
    }
    __syncthreads();
    if (!active) return;
    for (int32_t t = lane; t < nd * nn; t += 64) {
        const int32_t d = t / nn, e = t - d * nn;
        // the group of block d is [lo, end) of the list (ordered by block);
        // its values are loaded four at a time and added in candidate order
        int32_t lo, end;
        if (starts) {
            lo = sMo[w][d];
            end = sMo[w][d + 1];
        } else {
            int32_t hi = cc;
            lo = 0;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (sDw[sJw[mid]] < d) lo = mid + 1;
                else hi = mid;
            }
            end = lo;
            hi = cc;
            while (end < hi) {
                const int32_t mid = (end + hi) >> 1;
                if (sDw[sJw[mid]] <= d) end = mid + 1;
                else hi = mid;
            }
        }
        auto src = [&](int32_t g) { return val[(int64_t)(sKw[sJw[g]] & ~kFirst) * nn + e]; };
        double acc = 0.0;
        int32_t g = lo;
        for (; g + 4 <= end; g += 4) {
            const double v0 = src(g), v1 = src(g + 1), v2 = src(g + 2), v3 = src(g + 3);
            acc += v0; acc += v1; acc += v2; acc += v3;
        }
        for (; g < end; ++g) acc += src(g);
        valc[(int64_t)(base + d) * nn + e] = acc;
    }
}

// Thread-per-coarse-row Galerkin product for short candidate lists.  The
// distinct coarse columns are kept sorted (slot layout [slot][thread] in
// LDS); PASS 0 counts them, PASS 1 (scalar values only, n = 1) writes the
// columns and the sums, added in candidate order like k_rap.  The slots per
// thread set the LDS of a workgroup and so how many fit on a CU.  Most rows
// need few: with LIST false the kernel takes every row with CAP slots and
// leaves a row that needs more to a LIST launch with more slots, which runs
// over the rows queued in longq (*nlong of them).  PASS 0 queues a row at its
// (CAP+1)-th distinct column; PASS 1 skips the rows whose count exceeds CAP,
// which k_queue_long queued from the counts.
template <int PASS, int CAP, bool LIST>
__global__ __launch_bounds__(kRapSmallTpb) void k_rap_small(int32_t nc, const int32_t *__restrict__ aptr,
                                                            const int32_t *__restrict__ amem,
                                                            const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ col,
                                                            const double *__restrict__ w,
                                                            const int32_t *__restrict__ agg, int32_t *cnt,
                                                            const int32_t *__restrict__ rpc, int32_t *colc,
                                                            double *wc, int32_t *longq, int32_t *nlong) {
    __shared__ int32_t sJ[CAP * kRapSmallTpb];
    __shared__ double sS[PASS ? CAP * kRapSmallTpb : 1];
    const int t = threadIdx.x;
    const int32_t rows = LIST ? *nlong : nc;
    for (int32_t q = blockIdx.x * kRapSmallTpb + t; q < rows; q += gridDim.x * kRapSmallTpb) {
        const int32_t I = LIST ? longq[q] : q;
        if (PASS == 1 && !LIST && rpc[I + 1] - rpc[I] > CAP) continue;
        int nd = 0;
        bool over = false;
        for (int32_t m = aptr[I]; m < aptr[I + 1] && !over; ++m) {
            const int32_t i = amem[m];
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
                const int32_t J = agg[col[k]];
                int p = 0;
                while (p < nd && sJ[p * kRapSmallTpb + t] < J) ++p;
                if (p < nd && sJ[p * kRapSmallTpb + t] == J) {
                    if (PASS) sS[p * kRapSmallTpb + t] += w[k];
                    continue;
                }
                if (PASS == 0 && !LIST && nd == CAP) { over = true; break; }
                for (int r = nd; r > p; --r) {
                    sJ[r * kRapSmallTpb + t] = sJ[(r - 1) * kRapSmallTpb + t];
                    if (PASS) sS[r * kRapSmallTpb + t] = sS[(r - 1) * kRapSmallTpb + t];
                }
                sJ[p * kRapSmallTpb + t] = J;
                if (PASS) sS[p * kRapSmallTpb + t] = w[k];
                ++nd;
            }
        }
        if (PASS == 0) {
            if (over) longq[atomicAdd(nlong, 1)] = I;
            else cnt[I] = nd;
            continue;
        }
        const int32_t base = rpc[I];
        for (int d = 0; d < nd; ++d) {
            colc[base + d] = sJ[d * kRapSmallTpb + t];
            wc[base + d] = sS[d * kRapSmallTpb + t];
        }
    }
}

__global__ void k_queue_long(int32_t nc, const int32_t *rpc, int32_t cap, int32_t *longq, int32_t *nlong) {
    const int32_t I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I < nc && rpc[I + 1] - rpc[I] > cap) longq[atomicAdd(nlong, 1)] = I;
}

__device__ inline int32_t bsearch_col(const int32_t *col, int32_t lo, int32_t hi, int32_t j) {
    hi -= 1;
    while (lo <= hi) {
        const int32_t mid = (lo + hi) >> 1;
        const int32_t v = col[mid];
        if (v == j) return mid;
        if (v < j) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

// L lanes per row, each taking every L-th entry
template <int L>
__global__ void k_mirror_search(int32_t N, const int32_t *rp, const int32_t *col, int32_t *mirror,
                                int32_t *dslot, int32_t *flag) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t i = (int32_t)(t / L), lane = (int32_t)(t - (int64_t)i * L);
    if (i >= N) return;
    for (int32_t k = rp[i] + lane; k < rp[i + 1]; k += L) {
        const int32_t j = col[k];
        const int32_t m = bsearch_col(col, rp[j], rp[j + 1], i);
        if (m < 0) atomicOr(flag, 16);
        mirror[k] = m < 0 ? k : m;
        if (j == i) dslot[i] = k;
    }
}

__global__ void k_sys_first(int32_t N, const int32_t *row_sys, int64_t *first) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (i == 0 || row_sys[i] != row_sys[i - 1]) first[row_sys[i]] = i;
}

// ------------------------------------------------------------------ coarsest
// One workgroup per system: dense matrix of the system's rows, then
// Gauss-Jordan with partial pivoting in global memory (m = rows * n, small).
template <int n>
__global__ __launch_bounds__(256) void k_coarse_inverse(const int32_t *rp, const int32_t *col, const double *val,
                                                        const int64_t *roff_blk, const int64_t *off,
                                                        const int32_t *msz, double *work, double *inv,
                                                        double *invT, int32_t *flag) {
    const int s = blockIdx.x;
    const int m = msz[s];
    const int64_t r0 = roff_blk[s];               // first block row of the system
    double *a = work + off[s];
    double *x = inv + off[s];
    __shared__ int piv_row;
    __shared__ double piv_val;
    for (int64_t e = threadIdx.x; e < (int64_t)m * m; e += blockDim.x) {
        a[e] = 0.0;
        x[e] = ((e / m) == (e % m)) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int nb = m / n;
    for (int bi = threadIdx.x; bi < nb; bi += blockDim.x) {
        const int64_t i = r0 + bi;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int64_t bj = col[k] - r0;
            for (int r = 0; r < n; ++r)
                for (int c = 0; c < n; ++c)
                    a[((int64_t)bi * n + r) * m + bj * n + c] = val[(int64_t)k * n * n + r * n + c];
        }
    }
    __syncthreads();
    for (int k = 0; k < m; ++k) {
        if (threadIdx.x == 0) {
            int p = k;
            double pv = fabs(a[(int64_t)k * m + k]);
            for (int r = k + 1; r < m; ++r) {
                const double v = fabs(a[(int64_t)r * m + k]);
                if (v > pv) { pv = v; p = r; }
            }
            piv_row = p;
            piv_val = pv;
        }
        __syncthreads();
        if (!(piv_val > 0.0) || !isfinite(piv_val)) {
            if (threadIdx.x == 0) atomicOr(flag, 32);
            return;
        }
        const int p = piv_row;
        if (p != k) {
            for (int c = threadIdx.x; c < m; c += blockDim.x) {
                double t = a[(int64_t)k * m + c]; a[(int64_t)k * m + c] = a[(int64_t)p * m + c]; a[(int64_t)p * m + c] = t;
                t = x[(int64_t)k * m + c]; x[(int64_t)k * m + c] = x[(int64_t)p * m + c]; x[(int64_t)p * m + c] = t;
            }
        }
        __syncthreads();
        const double d = a[(int64_t)k * m + k];
        __syncthreads();
        for (int c = threadIdx.x; c < m; c += blockDim.x) {
            a[(int64_t)k * m + c] /= d;
            x[(int64_t)k * m + c] /= d;
        }
        __syncthreads();
        for (int64_t e = threadIdx.x; e < (int64_t)m * m; e += blockDim.x) {
            const int r = (int)(e / m), c = (int)(e % m);
            if (r == k) continue;
            const double f = a[(int64_t)r * m + k];
            if (c != k) a[e] -= f * a[(int64_t)k * m + c];
            x[e] -= f * x[(int64_t)k * m + c];
        }
        __syncthreads();
        for (int r = threadIdx.x; r < m; r += blockDim.x)
            if (r != k) a[(int64_t)r * m + k] = 0.0;
        __syncthreads();
    }
    for (int64_t e = threadIdx.x; e < (int64_t)m * m; e += blockDim.x) {
        const int r = (int)(e / m), c = (int)(e % m);
        invT[off[s] + (int64_t)c * m + r] = x[e];
    }
}

// The same Gauss-Jordan elimination with the augmented matrix [A | I] in LDS
// (row r at r * W, W = 2m + 1: the odd stride keeps a column's entries in
// different banks), for systems whose m fits.  One wavefront finds each
// pivot: the largest |a_rk| over rows r >= k, the first such row on ties
// (the serial scan's choice; NaN entries below the diagonal are passed over,
// a NaN diagonal makes the matrix singular).  Columns of A left of the pivot
// are dead once eliminated and are not updated, so each step is one pass
// that swaps and scales the pivot row, then one that eliminates the other
// rows; the inverse is the same as the global-memory kernel's.
template <int n>
__global__ __launch_bounds__(256) void k_coarse_inverse_lds(const int32_t *rp, const int32_t *col, const double *val,
                                                            const int64_t *roff_blk, const int64_t *off,
                                                            const int32_t *msz, double *inv, double *invT,
                                                            int32_t *flag) {
    extern __shared__ double ci_lds[];
    const int s = blockIdx.x;
    const int m = msz[s], W = 2 * m + 1;
    const int64_t r0 = roff_blk[s];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    constexpr int nw = 4;                          // wavefronts of the workgroup
    __shared__ int piv_row;
    __shared__ double piv_abs, piv_d;
    for (int e = t; e < m * W; e += blockDim.x) {
        const int r = e / W, j = e - r * W;
        ci_lds[e] = (j == m + r) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int nb = m / n;
    for (int bi = t; bi < nb; bi += blockDim.x) {
        const int64_t i = r0 + bi;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int bj = (int)(col[k] - r0);
            for (int r = 0; r < n; ++r)
                for (int c = 0; c < n; ++c)
                    ci_lds[(bi * n + r) * W + bj * n + c] = val[(int64_t)k * n * n + r * n + c];
        }
    }
    __syncthreads();
    for (int k = 0; k < m; ++k) {
        if (wv == 0) {
            double bv = -1.0;
            int br = m;
            for (int r = k + lane; r < m; r += 64) {
                const double v = fabs(ci_lds[r * W + k]);
                if (v > bv) { bv = v; br = r; }     // NaN is never greater
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const double ov = __shfl_xor(bv, o, 64);
                const int orow = __shfl_xor(br, o, 64);
                if (ov > bv || (ov == bv && orow < br)) { bv = ov; br = orow; }
            }
            if (lane == 0) {
                const double dk = ci_lds[k * W + k];
                piv_abs = dk != dk ? dk : bv;
                piv_row = br < m ? br : k;
                piv_d = ci_lds[(br < m ? br : k) * W + k];
            }
        }
        __syncthreads();
        const double pa = piv_abs;
        if (!(pa > 0.0) || !isfinite(pa)) {        // the same value in every thread
            if (t == 0) atomicOr(flag, 32);
            return;
        }
        const int p = piv_row;
        const double d = piv_d;
        for (int j = k + t; j < 2 * m; j += blockDim.x) {
            const double vp = ci_lds[p * W + j], vk = ci_lds[k * W + j];
            ci_lds[k * W + j] = vp / d;
            if (p != k) ci_lds[p * W + j] = vk;
        }
        __syncthreads();
        for (int r = wv; r < m; r += nw) {
            if (r == k) continue;
            const double f = ci_lds[r * W + k];
            for (int j = k + 1 + lane; j < 2 * m; j += 64) ci_lds[r * W + j] -= f * ci_lds[k * W + j];
        }
        __syncthreads();
    }
    for (int e = t; e < m * m; e += blockDim.x) {
        const int r = e / m, c = e - r * m;
        const double v = ci_lds[r * W + m + c];
        inv[off[s] + e] = v;
        invT[off[s] + (int64_t)c * m + r] = v;
    }
}

// ------------------------------------------------------------------ renumbering
// Positions come top-down from the aggregation tree: the rows of coarse row
// I' (new numbering) take the contiguous range start[I'] .. start[I'+1),
// in their previous relative order.  Rows that share an aggregate at any
// level therefore sit next to each other, so the x gathers of the block
// kernels stay within a few cache lines.
__global__ void k_pos_counts(int32_t nc, const int32_t *aptr, const int32_t *pos_c, int32_t *cnt) {
    const int32_t I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I < nc) cnt[pos_c[I]] = aptr[I + 1] - aptr[I];
}

__global__ void k_pos_assign(int32_t nc, const int32_t *aptr, const int32_t *amem, const int32_t *pos_c,
                             const int32_t *start, int32_t *pos_f) {
    const int32_t I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    const int32_t s0 = start[pos_c[I]];
    for (int32_t q = aptr[I]; q < aptr[I + 1]; ++q) pos_f[amem[q]] = s0 + (q - aptr[I]);
}

__global__ void k_invert(int32_t N, const int32_t *pos, int32_t *ip) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) ip[pos[i]] = i;
}

__global__ void k_perm_len(int32_t N, const int32_t *ip, const int32_t *rp, int32_t *len) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) len[i] = rp[ip[i] + 1] - rp[ip[i]];
}

// new row i' = old row ip[i'], columns renamed by pos and sorted; sk = old slot
// Row i' of the renumbered pattern is row ip[i'] of the old one with its
// columns renamed through pos and sorted; sk gives each new slot's old slot.
// Rows of up to MAXL blocks are ranked in registers (the columns of a row are
// distinct, so each entry's rank is the number of smaller columns); longer
// rows fall back to an insertion sort in place.
template <int MAXL>
__global__ void k_perm_rows(int32_t N, const int32_t *ip, const int32_t *pos, const int32_t *rp, const int32_t *col,
                            const int32_t *rpn, int32_t *coln, int32_t *sk) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t o = ip[i], b = rpn[i], len = rp[o + 1] - rp[o];
    if (len <= MAXL) {
        const int32_t r0 = rp[o];
        int32_t c[MAXL];
#pragma unroll
        for (int e = 0; e < MAXL; ++e) c[e] = e < len ? pos[col[r0 + e]] : INT32_MAX;
#pragma unroll
        for (int e = 0; e < MAXL; ++e) {
            if (e < len) {
                int32_t q = 0;
#pragma unroll
                for (int f = 0; f < MAXL; ++f) q += c[f] < c[e] ? 1 : 0;
                coln[b + q] = c[e];
                sk[b + q] = r0 + e;
            }
        }
        return;
    }
    for (int32_t e = 0; e < len; ++e) {
        const int32_t c = pos[col[rp[o] + e]], k = rp[o] + e;
        int32_t q = b + e - 1;
        while (q >= b && coln[q] > c) { coln[q + 1] = coln[q]; sk[q + 1] = sk[q]; --q; }
        coln[q + 1] = c;
        sk[q + 1] = k;
    }
}

// out block k = in block sk[k]; each thread moves V values: 4 or 2 when the
// block size allows (32- or 16-byte accesses), else a whole block row (n
// values; odd n, whose blocks do not align to 16 bytes)
template <int n>
__global__ void k_gather_blocks(int64_t nb, const int32_t *__restrict__ sk, const double *__restrict__ in,
                                double *__restrict__ out) {
    constexpr int nn = n * n, V = nn % 4 == 0 ? 4 : (nn % 2 == 0 ? 2 : n);
    typedef double dv __attribute__((ext_vector_type(V)));
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nb * (nn / V)) return;
    const int64_t k = g / (nn / V);
    const int64_t e = (g - k * (nn / V)) * V;
    if constexpr (V == n && n % 2 == 1) {
        const double *src = in + (int64_t)sk[k] * nn + e;
        double v[n];
#pragma unroll
        for (int c = 0; c < n; ++c) v[c] = src[c];
#pragma unroll
        for (int c = 0; c < n; ++c) out[k * nn + e + c] = v[c];
    } else {
        *reinterpret_cast<dv *>(out + k * nn + e) = *reinterpret_cast<const dv *>(in + (int64_t)sk[k] * nn + e);
    }
}

// a[e] = sk[a[e]] for the non-negative entries (a slot map of the internal
// numbering turned into one of the caller's block CSR)
__global__ void k_compose_slots(int64_t m, const int32_t *sk, int32_t *a) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const int32_t v = a[e];
    if (v >= 0) a[e] = sk[v];
}

// out[i'] = map[ip[i']], renamed through pos_c when given
__global__ void k_perm_map(int32_t N, const int32_t *ip, const int32_t *map, const int32_t *pos_c, int32_t *out) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t v = map[ip[i]];
    out[i] = pos_c ? pos_c[v] : v;
}

__global__ void k_iota(int32_t N, int32_t *a) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) a[i] = i;
}

__global__ void k_perm_vec(int32_t N, int n, const int32_t *__restrict__ ip, const double *__restrict__ in,
                           double *__restrict__ out, int to_internal) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)N * n) return;
    const int64_t i = g / n;
    const int q = (int)(g - i * n);
    if (to_internal) out[g] = in[(int64_t)ip[i] * n + q];
    else out[(int64_t)ip[i] * n + q] = in[g];
}

// ------------------------------------------------------------------ DILU setup
// Two colours when the block graph is bipartite (the face graph of any hex
// mesh is): a union-find over the graph's edges in which every node keeps
// its parent and its parity relative to that parent, packed as
// 2 * parent + parity; an edge joins its ends with opposite parity.  A larger
// root hooks under a smaller one by compare-and-swap on the root's word, so
// every parent has a smaller index than its child and every find ends; an
// edge whose ends already share a root with equal parity closes an odd cycle
// and sets the flag (the general colouring below then runs).  A node's colour
// is its parity relative to the root of its component -- its smallest node --
// which is its distance parity from that node, whatever order the edges were
// joined in.  The words are read and written at device scope (L1 bypassed),
// so a thread sees the hooks that others made.
__device__ inline int32_t uf_load(const int32_t *a) {
    return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int32_t uf_find(int32_t *uf, int32_t u, int &par) {
    int p = 0;
    for (;;) {
        const int32_t w = uf_load(uf + u);
        const int32_t up = w >> 1;
        if (up == u) break;
        const int32_t w2 = uf_load(uf + up);
        const int32_t g = w2 >> 1;
        if (g == up) {                       // the parent is a root
            p ^= w & 1;
            u = up;
            break;
        }
        // path halving: point u at its grandparent (any ancestor with the
        // parity of the path to it is a valid parent, so racing writes agree)
        const int32_t pw = (w ^ w2) & 1;
        __hip_atomic_store(uf + u, 2 * g + pw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        p ^= pw;
        u = g;
    }
    par = p;
    return u;
}

__global__ void k_uf_init(int32_t N, int32_t *uf) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) uf[i] = 2 * i;
}

__global__ void k_uf_hook(int32_t N, const int32_t *rp, const int32_t *col, int32_t *uf, int32_t *flag) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        const int32_t j = col[k];
        if (j <= i) continue;                    // each edge once, from its smaller end
        for (;;) {                               // ends when joined: a failed swap means another root hooked
            int pu, pv;
            const int32_t ru = uf_find(uf, i, pu), rv = uf_find(uf, j, pv);
            if (ru == rv) {
                if (pu == pv) atomicOr(flag, 1);
                break;
            }
            const int32_t hi = max(ru, rv), lo = min(ru, rv);
            if (atomicCAS(uf + hi, 2 * hi, 2 * lo + (1 ^ pu ^ pv)) == 2 * hi) break;
        }
    }
}

__global__ void k_uf_colour(int32_t N, int32_t *uf, int32_t *colour, int32_t *counters) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int par;
    uf_find(uf, i, par);
    colour[i] = par;
    if (par) atomicMax(&counters[1], 1);
}

// Colouring: Jones-Plassmann rounds with a fixed hash priority; a node whose
// uncoloured neighbours all rank lower takes the smallest colour unused by
// its coloured neighbours (first fit).  Nodes selected in one round are
// never adjacent, so the result does not depend on scheduling.
__device__ inline uint32_t mix32(uint32_t x) {
    x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
    return x;
}
__device__ inline bool outranks(int32_t j, int32_t i) {
    const uint32_t hj = mix32((uint32_t)j), hi = mix32((uint32_t)i);
    return hj > hi || (hj == hi && j > i);
}

__global__ void k_jp_select(int32_t N, const int32_t *rp, const int32_t *col, const int32_t *colour, int32_t *sel) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int32_t s = colour[i] < 0 ? 1 : 0;
    for (int32_t k = rp[i]; s && k < rp[i + 1]; ++k) {
        const int32_t j = col[k];
        if (j != i && colour[j] < 0 && outranks(j, i)) s = 0;
    }
    sel[i] = s;
}

// counters[0]: nodes coloured, [1]: largest colour, [2]: colour overflow
__global__ void k_jp_assign(int32_t N, const int32_t *rp, const int32_t *col, const int32_t *sel, int32_t *colour,
                            int32_t *counters) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N || !sel[i]) return;
    uint64_t m0 = 0, m1 = 0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        const int32_t j = col[k];
        const int32_t cj = j == i ? -1 : colour[j];
        if (cj >= 0 && cj < 64) m0 |= 1ull << cj;
        else if (cj >= 64 && cj < 128) m1 |= 1ull << (cj - 64);
    }
    int32_t c;
    if (~m0) c = __ffsll((long long)~m0) - 1;
    else if (~m1) c = 64 + __ffsll((long long)~m1) - 1;
    else { atomicOr(&counters[2], 1); c = 127; }
    colour[i] = c;
    atomicAdd(&counters[0], 1);
    atomicMax(&counters[1], c);
}

// rows ordered by (colour, index): per-block colour histograms, a scan in
// colour-major order, then in-block ranks
constexpr int kColourBlock = 256;
constexpr int kMaxColours = 128;

__global__ __launch_bounds__(kColourBlock) void k_colour_hist(int32_t N, int32_t ncol, int32_t nblk,
                                                              const int32_t *colour, int32_t *hist) {
    __shared__ int32_t hsh[kMaxColours];
    for (int c = threadIdx.x; c < kMaxColours; c += kColourBlock) hsh[c] = 0;
    __syncthreads();
    const int32_t i = blockIdx.x * kColourBlock + threadIdx.x;
    if (i < N) atomicAdd(&hsh[colour[i]], 1);
    __syncthreads();
    for (int c = threadIdx.x; c < ncol; c += kColourBlock) hist[(int64_t)c * nblk + blockIdx.x] = hsh[c];
}

__global__ __launch_bounds__(kColourBlock) void k_colour_place(int32_t N, int32_t nblk, const int32_t *colour,
                                                               const int32_t *off, int32_t *rows) {
    __shared__ int32_t sc[kColourBlock];
    const int32_t i = blockIdx.x * kColourBlock + threadIdx.x;
    sc[threadIdx.x] = i < N ? colour[i] : -1;
    __syncthreads();
    if (i >= N) return;
    const int32_t c = sc[threadIdx.x];
    int32_t rank = 0;
    for (int t = 0; t < (int)threadIdx.x; ++t) rank += sc[t] == c ? 1 : 0;
    rows[off[(int64_t)c * nblk + blockIdx.x] + rank] = i;
}

__global__ void k_colour_starts(int32_t ncol, int32_t nblk, const int32_t *off, int32_t *starts) {
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncol) starts[c] = off[(int64_t)c * nblk];
}

// E_i = A_ii - sum_{colour(j) < c} A_ij E_j^{-1} A_ji for the rows of colour c
template <int n>
__global__ __launch_bounds__(128) void k_dilu_setup(const int32_t *rows, int32_t cnt, int c, const int32_t *rp,
                                                    const int32_t *col,
                             const int32_t *mirror, const int32_t *dslot, const double *val,
                             const int32_t *colour, double *Einv, int32_t *bad) {
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= cnt) return;
    constexpr int nn = n * n;
    const int32_t i = rows[q];
    double E[n][2 * n];
    const double *Aii = val + (int64_t)dslot[i] * nn;
#pragma unroll
    for (int r = 0; r < n; ++r)
#pragma unroll
        for (int cc = 0; cc < n; ++cc) E[r][cc] = Aii[r * n + cc];
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        const int32_t j = col[k];
        if (j == i || colour[j] >= c) continue;
        const double *Aij = val + (int64_t)k * nn, *Aji = val + (int64_t)mirror[k] * nn;
        const double *Ej = Einv + (int64_t)j * nn;
        double T[n][n];
#pragma unroll
        for (int r = 0; r < n; ++r)
#pragma unroll
            for (int cc = 0; cc < n; ++cc) {
                double a = 0.0;
#pragma unroll
                for (int m = 0; m < n; ++m) a += Aij[r * n + m] * Ej[m * n + cc];
                T[r][cc] = a;
            }
#pragma unroll
        for (int r = 0; r < n; ++r)
#pragma unroll
            for (int cc = 0; cc < n; ++cc) {
                double a = 0.0;
#pragma unroll
                for (int m = 0; m < n; ++m) a += T[r][m] * Aji[m * n + cc];
                E[r][cc] -= a;
            }
    }
#pragma unroll
    for (int r = 0; r < n; ++r)
#pragma unroll
        for (int cc = 0; cc < n; ++cc) E[r][n + cc] = (r == cc) ? 1.0 : 0.0;
    const bool ok = gj_inverse<n>(E);
    if (!ok) atomicMin(bad, i);
    double *out = Einv + (int64_t)i * nn;
#pragma unroll
    for (int r = 0; r < n; ++r)
#pragma unroll
        for (int cc = 0; cc < n; ++cc) out[r * n + cc] = ok ? E[r][n + cc] : 0.0;
}

// Block ILU(0), rows of colour c (earlier colours are factored): the order is
// colour first, then row index.  F holds A's pattern; on entry row i holds
// A_i*, on exit the unscaled factor: F_ik = L_ik U_kk before the diagonal,
// U_ij from it on, so that M = L U = (E + F_lower) E^{-1} (E + F_upper) with
// E = diag(U).  The lower neighbours k are eliminated in increasing order:
// F_ij -= F_ik E_k^{-1} F_kj for every j of row i after k that row k holds
// (updates outside the pattern are dropped).  Row i is written only by its
// own thread; rows of earlier colours are final and only read.
template <int n>
__global__ __launch_bounds__(64) void k_ilu_setup(const int32_t *rows, int32_t cnt, int c, const int32_t *rp,
                                                  const int32_t *col,
                            const int32_t *dslot, const int32_t *colour, double *F, double *Einv, int32_t *bad) {
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= cnt) return;
    constexpr int nn = n * n;
    const int32_t i = rows[q];
    const int32_t b = rp[i], e = rp[i + 1];
    int32_t pc = -1, pj = -1;                      // last eliminated (colour, row)
    for (;;) {
        int32_t ks = -1, kc = 0, kk = 0;
        for (int32_t s = b; s < e; ++s) {          // next lower neighbour in order
            const int32_t j = col[s], cj = colour[j];
            if (cj >= c || cj < pc || (cj == pc && j <= pj)) continue;
            if (ks < 0 || cj < kc || (cj == kc && j < kk)) { ks = s; kc = cj; kk = j; }
        }
        if (ks < 0) break;
        pc = kc; pj = kk;
        double Lk[n][n];                           // F_ik E_k^{-1}
        const double *Fik = F + (int64_t)ks * nn, *Ek = Einv + (int64_t)kk * nn;
#pragma unroll
        for (int r = 0; r < n; ++r)
#pragma unroll
            for (int cc = 0; cc < n; ++cc) {
                double a = 0.0;
#pragma unroll
                for (int m = 0; m < n; ++m) a += Fik[r * n + m] * Ek[m * n + cc];
                Lk[r][cc] = a;
            }
        const int32_t kb = rp[kk], ke = rp[kk + 1];
        for (int32_t t = b; t < e; ++t) {
            const int32_t j = col[t], cj = colour[j];
            if (cj < kc || (cj == kc && j <= kk)) continue;     // j not after k
            int32_t kj = -1;
            for (int32_t u = kb; u < ke; ++u)
                if (col[u] == j) { kj = u; break; }
            if (kj < 0) continue;
            const double *Fkj = F + (int64_t)kj * nn;
            double *Fij = F + (int64_t)t * nn;
#pragma unroll
            for (int r = 0; r < n; ++r)
#pragma unroll
                for (int cc = 0; cc < n; ++cc) {
                    double a = 0.0;
#pragma unroll
                    for (int m = 0; m < n; ++m) a += Lk[r][m] * Fkj[m * n + cc];
                    Fij[r * n + cc] -= a;
                }
        }
    }
    double E[n][2 * n];
    const double *Fii = F + (int64_t)dslot[i] * nn;
#pragma unroll
    for (int r = 0; r < n; ++r)
#pragma unroll
        for (int cc = 0; cc < n; ++cc) {
            E[r][cc] = Fii[r * n + cc];
            E[r][n + cc] = (r == cc) ? 1.0 : 0.0;
        }
    const bool ok = gj_inverse<n>(E);
    if (!ok) atomicMin(bad, i);
    double *out = Einv + (int64_t)i * nn;
#pragma unroll
    for (int r = 0; r < n; ++r)
#pragma unroll
        for (int cc = 0; cc < n; ++cc) out[r * n + cc] = ok ? E[r][n + cc] : 0.0;
}

}  // namespace

// ====================================================================== host
#define NSWITCH(n, F, ...)                                                \
    switch (n) {                                                          \
        case 1: F<1>(__VA_ARGS__); break;                                 \
        case 2: F<2>(__VA_ARGS__); break;                                 \
        case 3: F<3>(__VA_ARGS__); break;                                 \
        case 4: F<4>(__VA_ARGS__); break;                                 \
        case 5: F<5>(__VA_ARGS__); break;                                 \
        default: cbs_throw(CBS_ERR_ARG, "bdim must be 1..5");             \
    }

namespace {

template <int n>
void blockinv_n(int32_t N, const int32_t *dslot, const double *val, double *Dinv, int32_t *bad, hipStream_t st) {
    if (N > 0)
        hipLaunchKernelGGL(k_blockinv<n>, dim3(cdiv(N, kInvThreads)), dim3(kInvThreads), 0, st, N, dslot, val, Dinv,
                           bad);
}
template <int n>
void transpose_n(int64_t nb, const int32_t *mirror, const double *in, double *out, hipStream_t st) {
    const int64_t tot = nb * n * n;
    if (tot > 0) hipLaunchKernelGGL(k_block_transpose<n>, dim3(cdiv(tot, 256)), dim3(256), 0, st, nb, mirror, in, out);
}
template <int n>
void strength_n(int32_t N, const int32_t *rp, const int32_t *col, const int32_t *mirror, const int32_t *dslot,
                const double *val, int64_t nnzb, double *df, double *w, hipStream_t st) {
    DArr<double> nrm(nnzb > 0 ? nnzb : 1);
    if (nnzb > 0) hipLaunchKernelGGL(k_block_frob<n>, dim3(cdiv(nnzb, 256)), dim3(256), 0, st, nnzb, val, nrm.get());
    hipLaunchKernelGGL(k_diag_norm, dim3(cdiv(N, 256)), dim3(256), 0, st, N, dslot, nrm.get(), df);
    if (lanes_for(N, nnzb) <= 8) {
        hipLaunchKernelGGL(k_strength, dim3(cdiv(N, 256)), dim3(256), 0, st, N, rp, col, mirror, nrm.get(), df, w);
    } else {
        hipLaunchKernelGGL(k_strength_lanes<16>, dim3(cdiv((int64_t)N * 16, 256)), dim3(256), 0, st, N, rp, col,
                           mirror, nrm.get(), df, w);
    }
}
template <int n>
void rap_n(int pass, int32_t nc, int32_t cap, const int32_t *aptr, const int32_t *amem, const int32_t *rp,
           const int32_t *col, const double *val, const int32_t *agg, int32_t *cnt, const int32_t *rpc, int32_t *colc,
           double *valc, int32_t *flag, hipStream_t st) {
    // at most 48 KB of LDS per workgroup: fewer wavefronts for long lists
    const int waves = std::max(1, std::min(kRapWaves, (int)(49152 / (12 * (size_t)cap))));
    const dim3 g(cdiv(nc, waves)), b(64 * waves);
    const size_t lds = sizeof(int32_t) * 3 * (size_t)cap * waves;
    if (pass == 0)
        hipLaunchKernelGGL((k_rap<n, 0>), g, b, lds, st, nc, cap, aptr, amem, rp, col, val, agg, cnt, rpc, colc, valc,
                           flag);
    else
        hipLaunchKernelGGL((k_rap<n, 1>), g, b, lds, st, nc, cap, aptr, amem, rp, col, val, agg, cnt, rpc, colc, valc,
                           flag);
}
template <int n>
void dilu_setup_n(const int32_t *rows, int32_t cnt, int c, const int32_t *rp, const int32_t *col, const int32_t *mirror,
                  const int32_t *dslot, const double *val, const int32_t *colour, double *Einv, int32_t *bad,
                  hipStream_t st) {
    if (cnt > 0)
        hipLaunchKernelGGL(k_dilu_setup<n>, dim3(cdiv(cnt, 128)), dim3(128), 0, st, rows, cnt, c, rp, col, mirror, dslot,
                           val, colour, Einv, bad);
}
template <int n>
void ilu_setup_n(const int32_t *rows, int32_t cnt, int c, const int32_t *rp, const int32_t *col, const int32_t *dslot,
                 const int32_t *colour, double *F, double *Einv, int32_t *bad, hipStream_t st) {
    if (cnt > 0)
        hipLaunchKernelGGL(k_ilu_setup<n>, dim3(cdiv(cnt, 64)), dim3(64), 0, st, rows, cnt, c, rp, col, dslot, colour,
                           F, Einv, bad);
}
template <int n>
void gather_blocks_n(int64_t nb, const int32_t *sk, const double *in, double *out, hipStream_t st) {
    constexpr int nn = n * n, V = nn % 4 == 0 ? 4 : (nn % 2 == 0 ? 2 : n);
    const int64_t tot = nb * (nn / V);
    if (tot > 0) hipLaunchKernelGGL(k_gather_blocks<n>, dim3(cdiv(tot, 256)), dim3(256), 0, st, nb, sk, in, out);
}
// lds > 0: the augmented matrices of every system fit in that much LDS
template <int n>
void coarse_inverse_n(int32_t n_sys, const int32_t *rp, const int32_t *col, const double *val, const int64_t *roffb,
                      const int64_t *off, const int32_t *msz, double *work, double *inv, double *invT, int32_t *flag,
                      size_t lds, hipStream_t st) {
    if (lds > 0) {
        if (lds > 64 * 1024)
            HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_coarse_inverse_lds<n>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(k_coarse_inverse_lds<n>, dim3(n_sys), dim3(256), lds, st, rp, col, val, roffb, off, msz,
                           inv, invT, flag);
    } else {
        hipLaunchKernelGGL(k_coarse_inverse<n>, dim3(n_sys), dim3(256), 0, st, rp, col, val, roffb, off, msz, work,
                           inv, invT, flag);
    }
}

struct Graph {
    int32_t N;
    const int32_t *rp, *col;
    const double *w;
    int lanes;                  // lanes per row of the matching kernels (4, 8 or 16)
};

// launch a kernel templated on the lanes per row over N rows
#define LANES_LAUNCH(KER, LN, N, ...)                                                                        \
    do {                                                                                                     \
        const int ln_ = (LN);                                                                                \
        const dim3 gl_(cdiv((int64_t)(N) * ln_, 256)), bl_(256);                                            \
        if (ln_ == 4) hipLaunchKernelGGL(KER<4>, gl_, bl_, 0, st, __VA_ARGS__);                             \
        else if (ln_ == 8) hipLaunchKernelGGL(KER<8>, gl_, bl_, 0, st, __VA_ARGS__);                        \
        else hipLaunchKernelGGL(KER<16>, gl_, bl_, 0, st, __VA_ARGS__);                                     \
    } while (0)

// one pass of handshake matching -> agg (size N); the aggregate count is left
// on the device in *nc (N > 0; not read back here)
void match_pass(cbs_system *h, const Graph &g, const int32_t *row_sys, const int32_t *sys_frozen, int32_t *agg,
                int32_t *nc) {
    hipStream_t st = h->stream;
    const int32_t N = g.N;
    DArr<int32_t> partner(N), cand(N), rep(N), root(N + 1);
    const dim3 G(cdiv(N, 256)), B(256);
    hipLaunchKernelGGL(k_match_init, G, B, 0, st, N, row_sys, sys_frozen, partner.get());
    for (int r = 0; r < kMatchRounds; ++r) {
        LANES_LAUNCH(k_match_pick, g.lanes, N, N, g.rp, g.col, g.w, partner.get(), cand.get());
        hipLaunchKernelGGL(k_match_confirm, G, B, 0, st, N, cand.get(), partner.get());
    }
    LANES_LAUNCH(k_match_rep, g.lanes, N, N, g.rp, g.col, g.w, partner.get(), rep.get(), root.get());
    LAUNCHCHK();
    scan_exclusive(root.get(), root.get(), N, st);
    hipLaunchKernelGGL(k_match_assign, G, B, 0, st, N, rep.get(), root.get(), agg, nc);
    LAUNCHCHK();
}

// Member lists of each aggregate (ascending) of a map of N rows onto at most
// N aggregates, sized for N so that they are built before the aggregate
// count comes back: past the last aggregate every aptr entry holds N.  The
// largest candidate list of the Galerkin product over the graph rp (the
// summed row lengths of an aggregate's members) goes to *maxc, which must
// hold 0.
void build_members(cbs_system *h, int32_t N, const int32_t *agg, DArr<int32_t> &aptr, DArr<int32_t> &amem,
                   const int32_t *rp, int32_t *maxc) {
    hipStream_t st = h->stream;
    aptr.alloc(N + 1);
    amem.alloc(N > 0 ? N : 1);
    DArr<int32_t> fill(N + 1), len(N + 1);
    hipLaunchKernelGGL(k_fill_int, dim3(cdiv(N + 1, 256)), dim3(256), 0, st, aptr.get(), (int64_t)N + 1, 0);
    hipLaunchKernelGGL(k_fill_int, dim3(cdiv(N + 1, 256)), dim3(256), 0, st, len.get(), (int64_t)N + 1, 0);
    hipLaunchKernelGGL(k_count_members_len, dim3(cdiv(N, 256)), dim3(256), 0, st, N, agg, rp, aptr.get(), len.get());
    hipLaunchKernelGGL(k_max_into, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(N, 256), 256))), dim3(256), 0, st,
                       (int64_t)N, len.get(), maxc);
    LAUNCHCHK();
    scan_exclusive(aptr.get(), aptr.get(), N, st);
    HIPCHK(hipMemcpyAsync(fill.get(), aptr.get(), sizeof(int32_t) * (N + 1), hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_fill_members, dim3(cdiv(N, 256)), dim3(256), 0, st, N, agg, fill.get(), amem.get());
    hipLaunchKernelGGL(k_sort_members, dim3(cdiv(N, 256)), dim3(256), 0, st, N, aptr.get(), amem.get());
    LAUNCHCHK();
}

// Galerkin pattern + values of the next level.  n_blk = block size of `val`.
// Returns the coarse block count when it builds the pattern, else -1.
// maxc: the largest candidate list when known (else < 0: found and read
// back here).  nz_bound >= 0: a bound on the coarse block count; the pattern
// is then sized for it and its count not read back (nz_bound is returned),
// and a candidate overflow sets bit 8 of *late_flag, which the caller reads
// later.
int32_t rap_build(cbs_system *h, int n_blk, int32_t nc, const int32_t *aptr, const int32_t *amem, const int32_t *rp,
                  const int32_t *col, const double *val, const int32_t *agg, DArr<int32_t> &rpc, DArr<int32_t> &colc,
                  DArr<double> &valc, bool pattern, int32_t maxc = -1, int64_t nz_bound = -1,
                  int32_t *late_flag = nullptr) {
    hipStream_t st = h->stream;
    const bool late = nz_bound >= 0 && late_flag;
    int32_t *flag = late ? late_flag : h->dflag.get();
    if (!late) hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, h->dflag.get(), (int64_t)2, 0);
    if (maxc < 0) {
        // largest candidate list of the level -> LDS per wavefront
        hipLaunchKernelGGL(k_rap_maxc, dim3(cdiv(nc, 256)), dim3(256), 0, st, nc, aptr, amem, rp, h->dflag.get() + 1);
        LAUNCHCHK();
        maxc = read_int(h->dflag.get() + 1, st);
    }
    if (maxc > kRapCap)
        cbs_throw(CBS_ERR_ARG, "a coarse row gathers " + std::to_string(maxc) + " blocks (limit " +
                                   std::to_string(kRapCap) + "); lower match_passes");
    int32_t cap = 64;
    while (cap < maxc) cap *= 2;
    // maxc bounds the distinct columns too, so short lists fit the slots; a
    // thread per row only pays when there are many rows (few rows with long
    // lists are faster a wavefront each)
    const bool many = nc >= kRapSmallRows;
    const bool small = many && maxc <= kRapSmall, small_count = many && maxc <= kRapSmallCount;
    const dim3 gs(cdiv(nc, kRapSmallTpb)), bs(kRapSmallTpb);
    int32_t nz = -1;
    // every row first takes the first launch's slots; when some row may need
    // more, the rows that do are queued for a second launch with the
    // kernel's limit (nlong[0]: rows of the counting pass, nlong[1]: of the
    // fill pass; both use longq, one after the other)
    const bool split_count = maxc > kRapCountSlots, split_fill = maxc > kRapSlots;
    const dim3 gl(std::min<int32_t>(cdiv(nc, kRapSmallTpb), kRapListGroups));
    DArr<int32_t> longq, nlong;
    if ((split_count || split_fill) && small_count && nc > 0) {
        longq.alloc(nc);
        nlong.alloc(2);
        hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, nlong.get(), (int64_t)2, 0);
    }
    if (pattern) {
        rpc.alloc(nc + 1);
        if (small_count && nc > 0) {
            hipLaunchKernelGGL((k_rap_small<0, kRapCountSlots, false>), gs, bs, 0, st, nc, aptr, amem, rp, col,
                               nullptr, agg, rpc.get(), nullptr, nullptr, nullptr, longq.get(), nlong.get());
            if (split_count)
                hipLaunchKernelGGL((k_rap_small<0, kRapSmallCount, true>), gl, bs, 0, st, nc, aptr, amem, rp, col,
                                   nullptr, agg, rpc.get(), nullptr, nullptr, nullptr, longq.get(), nlong.get());
        } else
            NSWITCH(n_blk, rap_n, 0, nc, cap, aptr, amem, rp, col, val, agg, rpc.get(), nullptr, nullptr, nullptr,
                    flag, st);
        LAUNCHCHK();
        scan_exclusive(rpc.get(), rpc.get(), nc, st);
        if (late) {
            nz = (int32_t)nz_bound;
        } else {
            // flag and count side by side: one copy back
            hipLaunchKernelGGL(k_copy_int, dim3(1), dim3(1), 0, st, rpc.get() + nc, h->dflag.get() + 1);
            LAUNCHCHK();
            int32_t v[2];
            read_array(h->dflag.get(), 2, v, st);
            if (v[0] & 8) cbs_throw(CBS_ERR_ARG, "coarse row candidate overflow");
            nz = v[1];
        }
        colc.alloc(nz > 0 ? nz : 1);
        valc.alloc((size_t)(nz > 0 ? nz : 1) * n_blk * n_blk);
    }
    // the fill pass visits the candidates the counting pass (or the first
    // build of this pattern) already fitted into cap, so it cannot overflow
    // (the small fill follows the small count of this call)
    if (small && small_count && pattern && n_blk == 1 && nc > 0) {
        int32_t *nlong_fill = nlong.get() ? nlong.get() + 1 : nullptr;
        if (split_fill)
            hipLaunchKernelGGL(k_queue_long, dim3(cdiv(nc, 256)), dim3(256), 0, st, nc, rpc.get(), kRapSlots,
                               longq.get(), nlong_fill);
        hipLaunchKernelGGL((k_rap_small<1, kRapSlots, false>), gs, bs, 0, st, nc, aptr, amem, rp, col, val, agg,
                           nullptr, rpc.get(), colc.get(), valc.get(), longq.get(), nlong_fill);
        if (split_fill)
            hipLaunchKernelGGL((k_rap_small<1, kRapSmall, true>), gl, bs, 0, st, nc, aptr, amem, rp, col, val, agg,
                               nullptr, rpc.get(), colc.get(), valc.get(), longq.get(), nlong_fill);
    } else
        NSWITCH(n_blk, rap_n, 1, nc, cap, aptr, amem, rp, col, val, agg, nullptr, rpc.get(), colc.get(), valc.get(),
                flag, st);
    LAUNCHCHK();
    return nz;
}

// Aggregation of level L into L.agg / L.nc (composed matching passes).
PhaseTimer *g_pt = nullptr;
inline void gmark(const char *w) { if (g_pt) g_pt->mark(w); }

// Each pass leaves its aggregate count on the device; the members and the
// largest Galerkin candidate list that the next step needs are built before
// that count is read, so one read-back per pass brings both.  The
// aggregate graphs of the later passes are sized by the level's block count
// (a bound on theirs) rather than read back; a candidate overflow there sets
// bit 8 of *deferred.  Leaves L.agg, L.nc, L.maxc and the members
// L.agg_ptr / L.agg_mem.
void aggregate_level(cbs_system *h, Level &L, const int32_t *sys_frozen, int32_t *deferred) {
    hipStream_t st = h->stream;
    const int32_t N = L.N;
    const int n = h->n;
    const int passes = std::max(1, h->opt.match_passes);
    DArr<double> df(N), w(L.nnzb > 0 ? L.nnzb : 1);
    // device words: [2p] the count of pass p, [2p + 1] the candidate maximum
    // after it, [2 passes] a spare
    const int nw_ = 2 * passes + 1;
    DArr<int32_t> words((size_t)nw_);
    hipLaunchKernelGGL(k_fill_int, dim3(cdiv(nw_, 64)), dim3(64), 0, st, words.get(), (int64_t)nw_, 0);
    NSWITCH(n, strength_n, N, L.rp, L.col, L.mirror, L.dslot, L.v64, L.nnzb, df.get(), w.get(), st);
    LAUNCHCHK();
    gmark("strength");
    L.agg.alloc(N);
    // the current graph (the level's, then each pass's aggregate graph) and
    // the last pass's map on it
    DArr<int32_t> grp, gcol, cur_rs;
    DArr<double> gw;
    const int32_t *cur_rp = L.rp, *cur_col = L.col, *cur_rowsys = L.row_sys.get();
    const double *cur_w = w.get();
    int32_t cur_N = N;
    int cur_lanes = lanes_for(N, L.nnzb);
    DArr<int32_t> aptr, amem;                      // members of the last pass's map on the current graph
    int32_t nc = 0, maxc = 0;
    for (int p = 0; p < passes; ++p) {
        DArr<int32_t> a(p > 0 ? cur_N : 1);
        int32_t *map = p == 0 ? L.agg.get() : a.get();
        Graph g{cur_N, cur_rp, cur_col, cur_w, cur_lanes};
        match_pass(h, g, cur_rowsys, sys_frozen, map, words.get() + 2 * p);
        if (p > 0) hipLaunchKernelGGL(k_compose, dim3(cdiv(N, 256)), dim3(256), 0, st, N, map, L.agg.get());
        LAUNCHCHK();
        // another pass works on this map's aggregate graph; after the last,
        // the level's Galerkin product on the composed map
        const bool more = p + 1 < passes;
        if (more) build_members(h, cur_N, map, aptr, amem, cur_rp, words.get() + 2 * p + 1);
        else build_members(h, N, L.agg.get(), L.agg_ptr, L.agg_mem, L.rp, words.get() + 2 * p + 1);
        int32_t v[2];
        read_array(words.get() + 2 * p, 2, v, st);
        nc = v[0];
        maxc = v[1];
        gmark(p == 0 ? "match1" : "match2");
        if (!more || nc <= 1) {
            if (more) {                            // stopped early: the level's members after all
                build_members(h, N, L.agg.get(), L.agg_ptr, L.agg_mem, L.rp, words.get() + 2 * passes);
                maxc = -1;                         // found again by the Galerkin product
            }
            break;
        }
        DArr<int32_t> nrp, ncol, nrs;
        DArr<double> nw;
        const int64_t bound = L.nnzb;
        rap_build(h, 1, nc, aptr.get(), amem.get(), cur_rp, cur_col, cur_w, map, nrp, ncol, nw, true, maxc, bound,
                  deferred);
        gmark("wrap");
        hipLaunchKernelGGL(k_zero_diag_w, dim3(cdiv(nc, 256)), dim3(256), 0, st, nc, nrp.get(), ncol.get(), nw.get());
        nrs.alloc(nc);
        hipLaunchKernelGGL(k_inherit_sys, dim3(cdiv(cur_N, 256)), dim3(256), 0, st, cur_N, map, cur_rowsys,
                           nrs.get());
        LAUNCHCHK();
        // the new graph becomes current (about twice the rows' degree)
        grp = std::move(nrp); gcol = std::move(ncol); gw = std::move(nw); cur_rs = std::move(nrs);
        cur_rp = grp.get(); cur_col = gcol.get(); cur_w = gw.get(); cur_rowsys = cur_rs.get();
        cur_lanes = lanes_for(cur_N, 2 * (int64_t)L.nnzb);
        cur_N = nc;
    }
    L.nc = nc;
    L.maxc = maxc;
}

// Multicolour ordering of level l (pattern only).
void colour_level(cbs_system *h, int l) {
    hipStream_t st = h->stream;
    Level &L = h->lev[l];
    const int32_t N = L.N;
    const dim3 G(cdiv(N, 256)), B(256);
    L.colour.alloc(N > 0 ? N : 1);
    DArr<int32_t> sel(N > 0 ? N : 1), cnt(4);
    HIPCHK(hipMemsetAsync(cnt.get(), 0, sizeof(int32_t) * 4, st));
    // two colours if the graph is bipartite (the packed words need N < 2^30)
    bool bipartite = false;
    if (N < (1 << 30)) {
        hipLaunchKernelGGL(k_uf_init, G, B, 0, st, N, sel.get());
        hipLaunchKernelGGL(k_uf_hook, G, B, 0, st, N, L.rp, L.col, sel.get(), cnt.get() + 3);
        hipLaunchKernelGGL(k_uf_colour, G, B, 0, st, N, sel.get(), L.colour.get(), cnt.get());
        LAUNCHCHK();
        bipartite = read_int(cnt.get() + 3, st) == 0;
    }
    int32_t done = bipartite ? N : 0;
    if (!bipartite) {
        hipLaunchKernelGGL(k_fill_int, G, B, 0, st, L.colour.get(), (int64_t)N, -1);
        HIPCHK(hipMemsetAsync(cnt.get(), 0, sizeof(int32_t) * 4, st));
    }
    for (int round = 0; done < N; ++round) {
        if (round >= 4096) cbs_throw(CBS_ERR_HIP, "colouring did not finish");
        hipLaunchKernelGGL(k_jp_select, G, B, 0, st, N, L.rp, L.col, L.colour.get(), sel.get());
        hipLaunchKernelGGL(k_jp_assign, G, B, 0, st, N, L.rp, L.col, sel.get(), L.colour.get(), cnt.get());
        LAUNCHCHK();
        if (round % 4 == 3) done = read_int(cnt.get(), st);
    }
    int32_t hc[3];
    HIPCHK(hipMemcpyAsync(hc, cnt.get(), sizeof(int32_t) * 3, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hc[2]) cbs_throw(CBS_ERR_ARG, "level " + std::to_string(l) + " needs more than 128 DILU colours; "
                                      "lower dilu_levels");
    const int32_t ncol = hc[1] + 1;
    const int32_t nblk = (int32_t)cdiv(N, kColourBlock);
    DArr<int32_t> hist((size_t)ncol * nblk + 1), starts(ncol + 1);
    hipLaunchKernelGGL(k_colour_hist, dim3(nblk), dim3(kColourBlock), 0, st, N, ncol, nblk, L.colour.get(), hist.get());
    LAUNCHCHK();
    scan_exclusive(hist.get(), hist.get(), (int64_t)ncol * nblk, st);
    L.rows_by_colour.alloc(N > 0 ? N : 1);
    hipLaunchKernelGGL(k_colour_place, dim3(nblk), dim3(kColourBlock), 0, st, N, nblk, L.colour.get(), hist.get(),
                       L.rows_by_colour.get());
    hipLaunchKernelGGL(k_colour_starts, dim3(cdiv(ncol, 64)), dim3(64), 0, st, ncol, nblk, hist.get(), starts.get());
    LAUNCHCHK();
    L.colour_off.assign(ncol + 1, 0);
    HIPCHK(hipMemcpyAsync(L.colour_off.data(), starts.get(), sizeof(int32_t) * ncol, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    L.colour_off[ncol] = N;
}

// E^{-1} of the DILU factorisation of level l, colour after colour (FP64).
void dilu_factor_level(cbs_system *h, int l) {
    hipStream_t st = h->stream;
    Level &L = h->lev[l];
    const int n = h->n;
    L.Einv.ensure((size_t)L.N * n * n);
    HIPCHK(hipMemsetAsync(h->dflag.get(), 0x7f, sizeof(int32_t), st));
    const int ncol = (int)L.colour_off.size() - 1;
    for (int c = 0; c < ncol; ++c) {
        const int32_t b0 = L.colour_off[c], cnt = L.colour_off[c + 1] - b0;
        NSWITCH(n, dilu_setup_n, L.rows_by_colour.get() + b0, cnt, c, L.rp, L.col, L.mirror, L.dslot, L.v64,
                L.colour.get(), L.Einv.get(), h->dflag.get(), st);
    }
    LAUNCHCHK();
    const int32_t bad = read_int(h->dflag.get(), st);
    if (bad != 0x7f7f7f7f)
        cbs_throw(CBS_ERR_SINGULAR, "singular DILU pivot at level " + std::to_string(l) + ", block row " +
                                        std::to_string(bad));
}

// Block ILU(0) of level l, colour after colour (FP64): the factor F in the
// level's BCSR pattern and E^{-1} in Einv.
void ilu_factor_level(cbs_system *h, int l) {
    hipStream_t st = h->stream;
    Level &L = h->lev[l];
    const int n = h->n;
    L.Einv.ensure((size_t)L.N * n * n);
    L.iluF.ensure((size_t)L.nnzb * n * n > 0 ? (size_t)L.nnzb * n * n : 1);
    HIPCHK(hipMemcpyAsync(L.iluF.get(), L.v64, sizeof(double) * (size_t)L.nnzb * n * n, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemsetAsync(h->dflag.get(), 0x7f, sizeof(int32_t), st));
    const int ncol = (int)L.colour_off.size() - 1;
    for (int c = 0; c < ncol; ++c) {
        const int32_t b0 = L.colour_off[c], cnt = L.colour_off[c + 1] - b0;
        NSWITCH(n, ilu_setup_n, L.rows_by_colour.get() + b0, cnt, c, L.rp, L.col, L.dslot, L.colour.get(),
                L.iluF.get(), L.Einv.get(), h->dflag.get(), st);
    }
    LAUNCHCHK();
    const int32_t bad = read_int(h->dflag.get(), st);
    if (bad != 0x7f7f7f7f)
        cbs_throw(CBS_ERR_SINGULAR, "singular ILU(0) pivot at level " + std::to_string(l) + ", block row " +
                                        std::to_string(bad));
}

// Values of the level's sliced copy (its pattern is built beforehand).
// f32flag: where the FP32 copy reports values it cannot hold (mixed only)
void level_sell(cbs_system *h, Level &L, bool mixed, int32_t *f32flag) {
    hipStream_t st = h->stream;
    const int n = h->n;
    const size_t tot = (size_t)L.sell.nent * n * n;
    L.sell.v64.ensure(tot > 0 ? tot : 1);
    if (mixed) L.sell.v32.ensure(tot > 0 ? tot : 1);
    sell_fill(n, L.sell, L.lazy_vals ? h->vals.get() : L.v64, L.sell.v64.get(), st, mixed ? L.sell.v32.get() : nullptr,
              f32flag);
}

std::vector<int64_t> level_sys_off(cbs_system *h, Level &L) {
    std::vector<int64_t> off(h->n_sys + 1, 0);
    if (h->n_sys == 1) {
        off[1] = L.N;
        return off;
    }
    DArr<int64_t> first(h->n_sys);
    hipLaunchKernelGGL(k_sys_first, dim3(cdiv(L.N, 256)), dim3(256), 0, h->stream, L.N, L.row_sys.get(), first.get());
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(off.data(), first.get(), sizeof(int64_t) * h->n_sys, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    off[h->n_sys] = L.N;
    return off;
}

void alloc_level_vectors(cbs_system *h, Level &L, bool mixed) {
    const size_t bytes = (size_t)L.N * h->n * (mixed ? sizeof(float) : sizeof(double));
    L.vb.ensure(bytes); L.vx.ensure(bytes); L.vr.ensure(bytes); L.vt.ensure(bytes);
    if (L.scaled) L.vc.ensure(bytes);
}

}  // namespace

void blockinv_level(cbs_system *h, int l, const double *vals, double *Dinv, int32_t *bad_slot,
                    const int32_t *dslot) {
    Level &L = h->lev[l];
    int32_t *slot = bad_slot ? bad_slot : h->dflag.get();
    HIPCHK(hipMemsetAsync(slot, 0x7f, sizeof(int32_t), h->stream));
    NSWITCH(h->n, blockinv_n, L.N, dslot ? dslot : L.dslot, vals, Dinv, slot, h->stream);
    LAUNCHCHK();
    if (bad_slot) return;                        // the caller checks later
    const int32_t bad = read_int(h->dflag.get(), h->stream);
    if (bad != 0x7f7f7f7f)
        cbs_throw(CBS_ERR_SINGULAR, "singular diagonal block at level " + std::to_string(l) + ", block row " +
                                        std::to_string(bad));
}

// Build (or, with reuse, refresh) the hierarchy.
void amg_setup(cbs_system *h) {
    hipStream_t st = h->stream;
    PhaseTimer pt(st, "setup");
    g_pt = &pt;
    struct Unset { ~Unset() { g_pt = nullptr; } } unset_;
    const cbs_options &o = h->opt;
    const int n = h->n;
    const bool mixed = o.precision == CBS_PRECISION_MIXED;
    const bool amg = o.precond == CBS_PREC_AMG;
    // cbs_setup keeps reuse_aggregates only when a complete hierarchy with the
    // same structural options exists
    const bool reuse = o.reuse_aggregates && amg && h->lev.size() > 1 && h->lev[0].agg.get() != nullptr;
    h->transposed_ready = false;
    // errors found by kernels are collected here and read back once at the
    // end: word 0 holds flag bits (8 aggregate-graph candidate overflow, 16
    // asymmetric coarse pattern, 32 singular coarsest matrix, 64 FP32
    // overflow), word 1 + l the first singular block row of level l
    DArr<int32_t> errs((size_t)std::max(1, o.max_levels) + 1);
    int32_t *deferred = errs.get();
    HIPCHK(hipMemsetAsync(errs.get(), 0x7f, sizeof(int32_t) * ((size_t)std::max(1, o.max_levels) + 1), st));
    HIPCHK(hipMemsetAsync(deferred, 0, sizeof(int32_t), st));

    if (!reuse) {
        h->lev.clear();
        h->renumbered = false;
        h->perm_sk.release();
    }
    pt.mark("free");
    if (h->lev.empty()) h->lev.emplace_back();
    Level &L0 = h->lev[0];
    if (!h->renumbered) {
        L0.N = h->N; L0.nnzb = h->nnzb;
        L0.rp = h->rp.get(); L0.col = h->col.get(); L0.mirror = h->mirror.get(); L0.dslot = h->dslot.get();
        L0.v64 = h->vals.get();
        if (!L0.row_sys.get()) build_row_sys(h, L0);
    } else {
        refresh_level0_values(h);
    }
    L0.sys_off = h->cell_off;
    pt.mark("level0");

    if (!amg) {
        // block Jacobi and symmetric Gauss-Seidel: level-0 block inverses;
        // Gauss-Seidel also colours level 0
        if (o.precond != CBS_PREC_NONE) {
            L0.Dinv.ensure((size_t)h->N * n * n);
            blockinv_level(h, 0, L0.v64, L0.Dinv.get());
        }
        const bool sgs = o.precond == CBS_PREC_SGS;
        if (sgs) colour_level(h, 0);
        h->lev.resize(1);
        sell_build(L0.N, L0.rp, L0.col, L0.sell, st, false, kSlice, sgs ? L0.rows_by_colour.get() : nullptr,
                   sgs ? &L0.colour_off : nullptr);
        level_sell(h, L0, false, nullptr);
        L0.sell.sched64 = choose_sched(n, L0.sell, false, L0.sell.v64.get(), o.schedule, st);
        L0.sell.sched64.split = row_split_for(L0.sell, L0.nnzb, o.row_split);
        h->op_complexity = 1.0;
        return;
    }

    DArr<int32_t> frozen(h->n_sys);
    std::vector<int32_t> hfrozen(h->n_sys);
    int l = 0;
    for (;; ++l) {
        Level &L = h->lev[l];
        if (L.sys_off.size() != (size_t)h->n_sys + 1) L.sys_off = level_sys_off(h, L);
        bool all_small = true;
        for (int s = 0; s < h->n_sys; ++s) {
            const int64_t Ns = L.sys_off[s + 1] - L.sys_off[s];
            hfrozen[s] = Ns <= o.coarse_max ? 1 : 0;
            all_small = all_small && hfrozen[s];
        }
        bool last = all_small || l + 1 >= o.max_levels;
        if (!last && !(reuse && L.agg.get() && (int)h->lev.size() > l + 1)) {
            HIPCHK(hipMemcpyAsync(frozen.get(), hfrozen.data(), sizeof(int32_t) * h->n_sys, hipMemcpyHostToDevice, st));
            aggregate_level(h, L, frozen.get(), deferred);
            pt.mark("agg" + std::to_string(l));
            // stall test over the systems still coarsening (frozen rows map 1:1)
            int64_t n_frozen = 0;
            for (int s = 0; s < h->n_sys; ++s)
                if (hfrozen[s]) n_frozen += L.sys_off[s + 1] - L.sys_off[s];
            const double active = (double)(L.N - n_frozen), active_c = (double)(L.nc - n_frozen);
            if (active_c > 0.97 * active) {                  // coarsening stalled
                L.agg.release(); L.nc = 0;
                last = true;
            } else {
                if ((int)h->lev.size() > l + 1) h->lev.resize(l + 1);
                h->lev.emplace_back();
                Level &C = h->lev[l + 1];
                Level &F = h->lev[l];
                C.N = F.nc;
                C.nnzb = rap_build(h, n, C.N, F.agg_ptr.get(), F.agg_mem.get(), F.rp, F.col, F.v64, F.agg.get(),
                                   C.o_rp, C.o_col, C.o_v64, true, F.maxc);
                C.rp = C.o_rp.get(); C.col = C.o_col.get(); C.v64 = C.o_v64.get();
                C.o_mirror.alloc(C.nnzb); C.o_dslot.alloc(C.N);
                C.mirror = C.o_mirror.get(); C.dslot = C.o_dslot.get();
                LANES_LAUNCH(k_mirror_search, lanes_for(C.N, C.nnzb), C.N, C.N, C.rp, C.col, C.mirror, C.dslot,
                             deferred);
                C.row_sys.alloc(C.N);
                hipLaunchKernelGGL(k_inherit_sys, dim3(cdiv(F.N, 256)), dim3(256), 0, st, F.N, F.agg.get(),
                                   F.row_sys.get(), C.row_sys.get());
                LAUNCHCHK();
                C.sys_off = level_sys_off(h, C);
                pt.mark("rap" + std::to_string(l));
                continue;
            }
        } else if (!last) {
            // reuse: refresh the values of level l+1 with the kept pattern
            Level &C = h->lev[l + 1];
            Level &F = h->lev[l];
            rap_build(h, n, C.N, F.agg_ptr.get(), F.agg_mem.get(), F.rp, F.col, F.v64, F.agg.get(), C.o_rp, C.o_col,
                      C.o_v64, false, F.maxc > 0 ? F.maxc : -1);
            continue;
        }
        // level l is the coarsest
        h->lev.resize(l + 1);
        h->lev[l].agg.release();
        h->lev[l].nc = 0;
        break;
    }
    const int nlev = (int)h->lev.size();
    auto level_uses_dilu = [&](int q) {
        return (o.smoother == CBS_SMOOTH_DILU || o.smoother == CBS_SMOOTH_SGS || o.smoother == CBS_SMOOTH_ILU0) &&
               (o.dilu_levels < 0 || q < o.dilu_levels) && q + 1 < nlev;
    };
    // a block-Jacobi level 0 keeps no values of its own in the internal
    // numbering: its copies and inverses read the caller's block CSR
    if (!reuse && o.renumber && nlev > 1) renumber_hierarchy(h, deferred, !level_uses_dilu(0));
    pt.mark("renumber");

    // sliced patterns of the solve phase: the full one of every smoothed level
    // (and level 0), the off-diagonal one of the mixed block-Jacobi levels;
    // new patterns share one read-back of their entry counts
    {
        // coloured levels first get their colours: their sliced copy holds
        // each colour's rows as one run of slices
        for (int q = 0; q + 1 < nlev; ++q)
            if (level_uses_dilu(q) && (!reuse || !h->lev[q].colour.get())) colour_level(h, q);
        pt.mark("colours");
        struct Pending { Level *L; Sell *S; bool od; bool coloured; };
        std::vector<Pending> todo;
        for (int q = 0; q < nlev; ++q) {
            Level &L = h->lev[q];
            const bool keep_sell = reuse && L.sell.N == L.N && L.sell.soff.get();
            const bool keep_sod = reuse && L.sod.N == L.N && L.sod.soff.get();
            if ((q == 0 || q + 1 < nlev) && !keep_sell)
                todo.push_back({&L, &L.sell, false, q + 1 < nlev && level_uses_dilu(q)});
            if (mixed && o.scaled_sweeps && q + 1 < nlev && !level_uses_dilu(q) && !keep_sod)
                todo.push_back({&L, &L.sod, true, false});
        }
        for (auto &t : todo)
            sell_pattern_begin(t.L->N, t.L->rp, t.L->col, *t.S, st, t.od, t.L == &h->lev[0] ? kSlice : kCoarseSlice,
                               t.coloured ? t.L->rows_by_colour.get() : nullptr,
                               t.coloured ? &t.L->colour_off : nullptr);
        for (size_t k0 = 0; k0 < todo.size(); k0 += kPinnedWords) {
            const size_t k1 = std::min(todo.size(), k0 + kPinnedWords);
            int32_t cnt[kPinnedWords];
            int32_t *w = pinned_words();
            for (size_t k = k0; k < k1; ++k) {   // one synchronisation per 64 patterns
                const Sell &S = *todo[k].S;
                HIPCHK(hipMemcpyAsync(w + (k - k0), S.soff.get() + S.nslices, sizeof(int32_t), hipMemcpyDeviceToHost,
                                      st));
            }
            HIPCHK(hipStreamSynchronize(st));
            for (size_t k = k0; k < k1; ++k) cnt[k - k0] = w[k - k0];
            for (size_t k = k0; k < k1; ++k)
                sell_pattern_finish(todo[k].L->rp, todo[k].L->col, *todo[k].S, cnt[k - k0], st, todo[k].od);
        }
        // the copies of a level 0 without its own values point into the caller's block CSR
        for (auto &t : todo)
            if (t.L->lazy_vals && t.S->nent > 0) {
                hipLaunchKernelGGL(k_compose_slots, dim3(cdiv(t.S->nent, 256)), dim3(256), 0, st, t.S->nent,
                                   h->perm_sk.get(), t.S->ssrc.get());
                LAUNCHCHK();
            }
        pt.mark("patterns");
    }

    // smoothers (FP64 inverses), FP32 copies, vectors
    int64_t nz_sum = 0;
    for (int q = 0; q < nlev; ++q) {
        Level &L = h->lev[q];
        nz_sum += L.nnzb;
        const bool coloured = level_uses_dilu(q);   // DILU, symmetric Gauss-Seidel or ILU(0)
        // ILU(0) runs the DILU sweeps on its own factor: it carries both flags
        L.dilu = q + 1 < nlev && coloured && (o.smoother == CBS_SMOOTH_DILU || o.smoother == CBS_SMOOTH_ILU0);
        L.ilu = L.dilu && o.smoother == CBS_SMOOTH_ILU0;
        L.sgs = q + 1 < nlev && coloured && o.smoother == CBS_SMOOTH_SGS;
        if (L.ilu) {
            ilu_factor_level(h, q);
        } else if (L.dilu) {
            dilu_factor_level(h, q);
        } else if (q + 1 < nlev) {                  // block Jacobi and Gauss-Seidel: D^{-1}
            L.Dinv.ensure((size_t)L.N * n * n);
            if (L.lazy_vals) blockinv_level(h, q, h->vals.get(), L.Dinv.get(), errs.get() + 1 + q, L.dslot_src.get());
            else blockinv_level(h, q, L.v64, L.Dinv.get(), errs.get() + 1 + q);
        }
        pt.mark("smoother" + std::to_string(q));
        L.scaled = mixed && o.scaled_sweeps && q + 1 < nlev && !L.dilu && !L.sgs;
        L.scaledT = false;
        if (L.scaled) {
            // the full and the row-scaled off-diagonal copy in one pass over the values
            const size_t tot = (size_t)L.sell.nent * n * n;
            L.sell.v64.ensure(tot > 0 ? tot : 1);
            L.sell.v32.ensure(tot > 0 ? tot : 1);
            L.sod.v32.ensure(L.sod.nent > 0 ? (size_t)L.sod.nent * n * n : 1);
            sell_fill_scaled(n, L.sell, L.sod, L.lazy_vals ? h->vals.get() : L.v64, L.Dinv.get(), L.sell.v64.get(),
                             L.sell.v32.get(), L.sod.v32.get(), deferred, st);
        } else {
            if (q == 0 || q + 1 < nlev) level_sell(h, L, mixed, deferred);
            L.sod = Sell();
        }
        if (L.ilu) {
            const size_t tot = (size_t)L.sell.nent * n * n;
            L.iluS64.ensure(tot > 0 ? tot : 1);
            if (mixed) L.iluS32.ensure(tot > 0 ? tot : 1);
            sell_fill(n, L.sell, L.iluF.get(), L.iluS64.get(), st, mixed ? L.iluS32.get() : nullptr, deferred);
        } else {
            L.iluF.release(); L.iluS64.release(); L.iluS32.release(); L.iluS64T.release(); L.iluS32T.release();
        }
        alloc_level_vectors(h, L, mixed);
        pt.mark("sell" + std::to_string(q));
    }
    {
        // schedules of the block-row kernels, tuned on level 0, used on every level
        Level &T0 = h->lev[0];
        const Sched s64 = choose_sched(n, T0.sell, false, T0.sell.v64.get(), o.schedule, st);
        const Sched s32 = mixed ? choose_sched(n, T0.sell, true, T0.sell.v32.get(), o.schedule, st) : Sched{4, 1};
        for (auto &L : h->lev) {
            L.sell.sched64 = L.sod.sched64 = s64;
            L.sell.sched32 = L.sod.sched32 = s32;
            L.sell.sched64.split = L.sell.sched32.split = row_split_for(L.sell, L.nnzb, o.row_split);
            L.sod.sched32.split = row_split_for(L.sod, L.nnzb - L.N, o.row_split);
        }
        pt.mark("autotune");
    }
    if (mixed) {
        // FP32 level values that overflow (flagged while the FP32 copies and
        // the row-scaled values were written): escalate the hierarchy to FP64
        if (read_int(deferred, st) & 64) {
            h->opt.precision = CBS_PRECISION_FP64;
            h->precision_fallback = true;
            for (int q = 0; q < nlev; ++q) alloc_level_vectors(h, h->lev[q], false);
        }
    }
    h->op_complexity = (double)nz_sum / (double)h->nnzb;

    // coarsest: dense inverse of each system
    Level &Lc = h->lev[nlev - 1];
    std::vector<int64_t> off(h->n_sys + 1, 0), roffb(h->n_sys), roff(h->n_sys);
    std::vector<int32_t> msz(h->n_sys);
    int32_t maxm = 0;
    for (int s = 0; s < h->n_sys; ++s) {
        const int64_t rows = Lc.sys_off[s + 1] - Lc.sys_off[s];
        const int64_t m = rows * n;
        if (m > 4096)
            cbs_throw(CBS_ERR_ARG, "coarsest system too large for the dense solve (" + std::to_string(m) +
                                       " unknowns); raise max_levels or lower coarse_max");
        msz[s] = (int32_t)m;
        roffb[s] = Lc.sys_off[s];
        roff[s] = Lc.sys_off[s] * n;
        off[s + 1] = off[s] + m * m;
        maxm = std::max<int32_t>(maxm, (int32_t)m);
    }
    Coarse &C = h->coarse;
    C.max_m = maxm;
    C.inv.ensure(off[h->n_sys] > 0 ? off[h->n_sys] : 1);
    C.invT.ensure(off[h->n_sys] > 0 ? off[h->n_sys] : 1);
    C.off.ensure(h->n_sys + 1); C.m.ensure(h->n_sys); C.roff.ensure(h->n_sys);
    DArr<int64_t> droffb(h->n_sys);
    // [A | I] of the largest system in LDS (beside the kernel's few static
    // words), else the elimination runs in global memory
    const size_t ci_lds = sizeof(double) * (size_t)maxm * (2 * (size_t)maxm + 1);
    const bool ci_in_lds = maxm > 0 && ci_lds + 1024 <= (size_t)h->lds_max;
    DArr<double> work(ci_in_lds ? 1 : (off[h->n_sys] > 0 ? off[h->n_sys] : 1));
    HIPCHK(hipMemcpyAsync(C.off.get(), off.data(), sizeof(int64_t) * (h->n_sys + 1), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(C.m.get(), msz.data(), sizeof(int32_t) * h->n_sys, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(C.roff.get(), roff.data(), sizeof(int64_t) * h->n_sys, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(droffb.get(), roffb.data(), sizeof(int64_t) * h->n_sys, hipMemcpyHostToDevice, st));
    NSWITCH(n, coarse_inverse_n, h->n_sys, Lc.rp, Lc.col, Lc.v64, droffb.get(), C.off.get(), C.m.get(), work.get(),
            C.inv.get(), C.invT.get(), deferred, ci_in_lds ? ci_lds : 0, st);
    LAUNCHCHK();
    // one read-back of every error the setup kernels recorded
    std::vector<int32_t> ev((size_t)nlev + 1);
    for (int32_t k0 = 0; k0 < nlev + 1; k0 += kPinnedWords)
        read_array(errs.get() + k0, std::min<int32_t>(kPinnedWords, nlev + 1 - k0), ev.data() + k0, st);
    if (ev[0] & 8) cbs_throw(CBS_ERR_ARG, "aggregate graph row candidate overflow");
    if (ev[0] & 16) cbs_throw(CBS_ERR_PATTERN, "coarse pattern is not symmetric");
    for (int q = 0; q + 1 < nlev; ++q)
        if (!h->lev[q].dilu && ev[1 + q] != 0x7f7f7f7f)
            cbs_throw(CBS_ERR_SINGULAR, "singular diagonal block at level " + std::to_string(q) + ", block row " +
                                            std::to_string(ev[1 + q]));
    if (ev[0] & 32) cbs_throw(CBS_ERR_SINGULAR, "coarsest-level matrix is singular");
    pt.mark("coarse");
}

// Transposed level values for the adjoint solve: A^T(i,j) = A(j,i)^T through
// the mirror map (a bit-exact permuted copy), D^{-T} = (D^{-1})^T.
void amg_build_transposed(cbs_system *h) {
    if (h->transposed_ready) return;
    hipStream_t st = h->stream;
    const int n = h->n;
    const bool mixed = h->opt.precision == CBS_PRECISION_MIXED;
    const int nlev = (int)h->lev.size();
    HIPCHK(hipMemsetAsync(h->dflag.get(), 0, sizeof(int32_t), st));
    for (int q = 0; q < nlev; ++q) {
        Level &L = h->lev[q];
        L.o_v64T.ensure((size_t)L.nnzb * n * n);
        L.v64T = L.o_v64T.get();
        // (a level 0 without its own values: A^T in the caller's slots, which
        // its copies' slot maps point to)
        if (L.lazy_vals) {
            NSWITCH(n, transpose_n, L.nnzb, h->mirror.get(), h->vals.get(), L.v64T, st);
        } else {
            NSWITCH(n, transpose_n, L.nnzb, L.mirror, L.v64, L.v64T, st);
        }
        if (L.sell.soff.get()) {
            const size_t tot = (size_t)L.sell.nent * n * n;
            L.sell.v64T.ensure(tot > 0 ? tot : 1);
            if (mixed) L.sell.v32T.ensure(tot > 0 ? tot : 1);
            sell_fill(n, L.sell, L.v64T, L.sell.v64T.get(), st, mixed ? L.sell.v32T.get() : nullptr, h->dflag.get());
        }
        if (L.Dinv.get()) {
            L.DinvT.ensure((size_t)L.N * n * n);
            NSWITCH(n, transpose_n, (int64_t)L.N, nullptr, L.Dinv.get(), L.DinvT.get(), st);
        }
        if (L.dilu) {
            // DILU of A^T in the same ordering has E' = E^T
            L.EinvT.ensure((size_t)L.N * n * n);
            NSWITCH(n, transpose_n, (int64_t)L.N, nullptr, L.Einv.get(), L.EinvT.get(), st);
        }
        if (L.ilu && L.sell.soff.get()) {
            // ILU(0) of A^T in the same ordering: M^T = (E^T + F_upper^T) E^{-T}
            // (E^T + F_lower^T) matches A^T on the pattern, so F' = F^T blockwise
            const size_t nb = (size_t)L.nnzb * n * n, tot = (size_t)L.sell.nent * n * n;
            DArr<double> FT(nb > 0 ? nb : 1);
            NSWITCH(n, transpose_n, L.nnzb, L.mirror, L.iluF.get(), FT.get(), st);
            L.iluS64T.ensure(tot > 0 ? tot : 1);
            if (mixed) L.iluS32T.ensure(tot > 0 ? tot : 1);
            sell_fill(n, L.sell, FT.get(), L.iluS64T.get(), st, mixed ? L.iluS32T.get() : nullptr, h->dflag.get());
        }
        if (mixed && L.scaled) {
            // row-scaled off-diagonal values of A^T: D_i^{-T} (A^T)_ij, j != i
            L.sod.v32T.ensure(L.sod.nent > 0 ? (size_t)L.sod.nent * n * n : 1);
            sell_scale(n, L.sod, L.v64T, L.DinvT.get(), L.sod.v32T.get(), h->dflag.get(), st);
        }
        LAUNCHCHK();
    }
    // FP32 cannot hold some scaled value: the transposed sweeps keep D^{-T}
    const bool overflow = read_int(h->dflag.get(), st) & 64;
    for (auto &L : h->lev) L.scaledT = mixed && L.scaled && !overflow;
    h->transposed_ready = true;
}

// Permute every level but the coarsest into the aggregation-tree order;
// pattern errors go to the flag word `deferred`.
void renumber_hierarchy(cbs_system *h, int32_t *deferred, bool lazy0) {
    hipStream_t st = h->stream;
    const int n = h->n;
    const int nlev = (int)h->lev.size();
    if (nlev < 2) return;
    std::vector<DArr<int32_t>> pos(nlev);
    {
        Level &C = h->lev[nlev - 1];
        pos[nlev - 1].alloc(C.N);
        hipLaunchKernelGGL(k_iota, dim3(cdiv(C.N, 256)), dim3(256), 0, st, C.N, pos[nlev - 1].get());
    }
    std::vector<DArr<int32_t>> new_aptr(nlev);
    for (int l = nlev - 2; l >= 0; --l) {
        Level &F = h->lev[l];
        const int32_t nc = F.nc;
        new_aptr[l].alloc(nc + 1);
        hipLaunchKernelGGL(k_pos_counts, dim3(cdiv(nc, 256)), dim3(256), 0, st, nc, F.agg_ptr.get(), pos[l + 1].get(),
                           new_aptr[l].get());
        LAUNCHCHK();
        scan_exclusive(new_aptr[l].get(), new_aptr[l].get(), nc, st);
        pos[l].alloc(F.N);
        hipLaunchKernelGGL(k_pos_assign, dim3(cdiv(nc, 256)), dim3(256), 0, st, nc, F.agg_ptr.get(), F.agg_mem.get(),
                           pos[l + 1].get(), new_aptr[l].get(), pos[l].get());
        LAUNCHCHK();
    }
    gmark("positions");
    for (int l = 0; l + 1 < nlev; ++l) {
        Level &L = h->lev[l];
        const int32_t N = L.N;
        const int64_t nnz = L.nnzb;
        const dim3 G(cdiv(N, 256)), B(256);
        DArr<int32_t> ip(N), rpn(N + 1), coln(nnz), sk(nnz), aggn(N), memn(N), rsn(N), mir(nnz), dsl(N);
        if (l == 0) gmark("alloc0");
        const bool lazy = l == 0 && lazy0;
        DArr<double> vn(lazy ? 0 : (size_t)nnz * n * n);
        hipLaunchKernelGGL(k_invert, G, B, 0, st, N, pos[l].get(), ip.get());
        hipLaunchKernelGGL(k_perm_len, G, B, 0, st, N, ip.get(), L.rp, rpn.get());
        LAUNCHCHK();
        scan_exclusive(rpn.get(), rpn.get(), N, st);
        if (l == 0)        // level 0: short rows (face neighbours)
            hipLaunchKernelGGL(k_perm_rows<16>, G, B, 0, st, N, ip.get(), pos[l].get(), L.rp, L.col, rpn.get(),
                               coln.get(), sk.get());
        else
            hipLaunchKernelGGL(k_perm_rows<32>, G, B, 0, st, N, ip.get(), pos[l].get(), L.rp, L.col, rpn.get(),
                               coln.get(), sk.get());
        if (!lazy) {
            NSWITCH(n, gather_blocks_n, nnz, sk.get(), L.v64, vn.get(), st);
        }
        hipLaunchKernelGGL(k_perm_map, G, B, 0, st, N, ip.get(), L.agg.get(), pos[l + 1].get(), aggn.get());
        hipLaunchKernelGGL(k_iota, G, B, 0, st, N, memn.get());
        hipLaunchKernelGGL(k_perm_map, G, B, 0, st, N, ip.get(), L.row_sys.get(), nullptr, rsn.get());
        LANES_LAUNCH(k_mirror_search, lanes_for(N, nnz), N, N, rpn.get(), coln.get(), mir.get(), dsl.get(), deferred);
        LAUNCHCHK();
        L.lazy_vals = lazy;
        if (lazy) {                                    // caller slots of the internal diagonal blocks
            L.dslot_src.alloc(N);
            HIPCHK(hipMemcpyAsync(L.dslot_src.get(), dsl.get(), sizeof(int32_t) * N, hipMemcpyDeviceToDevice, st));
            hipLaunchKernelGGL(k_compose_slots, G, B, 0, st, (int64_t)N, sk.get(), L.dslot_src.get());
            LAUNCHCHK();
        }
        if (l == 0) h->perm_sk = std::move(sk);
        L.o_rp = std::move(rpn); L.o_col = std::move(coln); L.o_v64 = std::move(vn);
        L.o_mirror = std::move(mir); L.o_dslot = std::move(dsl);
        L.rp = L.o_rp.get(); L.col = L.o_col.get(); L.v64 = lazy ? nullptr : L.o_v64.get();
        L.mirror = L.o_mirror.get(); L.dslot = L.o_dslot.get();
        L.agg = std::move(aggn); L.agg_ptr = std::move(new_aptr[l]); L.agg_mem = std::move(memn);
        L.row_sys = std::move(rsn);
        L.order = std::move(ip);
        if (l == 0) gmark("perm0");
    }
    h->renumbered = true;
}

// Level-0 values in the internal numbering after a coefficient update.
// (a level 0 without its own copy gets one here: the Galerkin product of
// level 1 in the re-setup reads the internal numbering)
void refresh_level0_values(cbs_system *h) {
    Level &L0 = h->lev[0];
    if (L0.lazy_vals) {
        L0.o_v64.ensure((size_t)h->nnzb * h->n * h->n);
        L0.v64 = L0.o_v64.get();
    }
    NSWITCH(h->n, gather_blocks_n, h->nnzb, h->perm_sk.get(), h->vals.get(), L0.o_v64.get(), h->stream);
    LAUNCHCHK();
}

void level0_values_into(cbs_system *h, double *out) {
    Level &L0 = h->lev[0];
    if (!L0.lazy_vals) {
        HIPCHK(hipMemcpyAsync(out, L0.v64, sizeof(double) * (size_t)h->nnzb * h->n * h->n, hipMemcpyDeviceToDevice,
                              h->stream));
        return;
    }
    NSWITCH(h->n, gather_blocks_n, h->nnzb, h->perm_sk.get(), h->vals.get(), out, h->stream);
    LAUNCHCHK();
}

// Caller numbering <-> internal numbering of a level-0 vector.
void permute_vec(cbs_system *h, const double *in, double *out, bool to_internal) {
    const int64_t m = (int64_t)h->N * h->n;
    if (m > 0)
        hipLaunchKernelGGL(k_perm_vec, dim3(cdiv(m, 256)), dim3(256), 0, h->stream, h->N, h->n, h->lev[0].order.get(),
                           in, out, to_internal ? 1 : 0);
    LAUNCHCHK();
}

// cbs_spmv: caller-numbered A or A^T (sliced copy built on first use)
void spmv_user(cbs_system *h, const double *x, double *y, bool transposed) {
    Sell &U = h->usell;
    const int n = h->n;
    const size_t tot = 0;
    (void)tot;
    if (!U.soff.get()) sell_build(h->N, h->rp.get(), h->col.get(), U, h->stream);
    const bool tune = !U.v64.get() && !U.v64T.get();
    const size_t nv = (size_t)U.nent * n * n;
    if (!transposed) {
        if (!U.v64.get()) {
            U.v64.alloc(nv > 0 ? nv : 1);
            sell_fill(n, U, h->vals.get(), U.v64.get(), h->stream);
        }
        if (tune) {
            U.sched64 = choose_sched(n, U, false, U.v64.get(), h->opt.schedule, h->stream);
            U.sched64.split = row_split_for(U, h->nnzb, h->opt.row_split);
        }
        launch_rows<double, double>(0, n, U.view(), U.v64.get(), x, nullptr, y, nullptr, 0.0, h->stream);
        return;
    }
    if (!U.v64T.get()) {
        h->valsT.alloc((size_t)h->nnzb * n * n);
        NSWITCH(n, transpose_n, h->nnzb, h->mirror.get(), h->vals.get(), h->valsT.get(), h->stream);
        LAUNCHCHK();
        U.v64T.alloc(nv > 0 ? nv : 1);
        sell_fill(n, U, h->valsT.get(), U.v64T.get(), h->stream);
        h->valsT.release();
    }
    launch_rows<double, double>(0, n, U.view(), U.v64T.get(), x, nullptr, y, nullptr, 0.0, h->stream);
}
