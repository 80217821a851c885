// convert.hip -- face-addressed LDU -> block CSR on the device, field
// packing, and the LDU-layout gradient.
//
// Sec. 2.3 (Alg. amgxFoam, Fig. block_amgx): the coupled matrix keeps the
// sparsity of the scalar problem; only the indices now address n x n blocks.
// The conversion is a permutation of whole blocks, so it is done as
//   pattern (once per topology): degree count -> scan -> placement -> per-row
//     sort by column (diagonal inline) -> slot maps for diag/upper/lower;
//   values (every coefficient update): vals[slot] = source block, copied
//     element for element (bit-exact), writes fully coalesced.
#include "cbs_internal.h"

#include <cstdlib>
#include <mutex>
#include <string>

#include <algorithm>

// ------------------------------------------------------------------ scan
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanThreads * kScanPer;

__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t *total) {
    __shared__ int32_t wsum[kScanThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int32_t o = __shfl_up(inc, d, 64);
        if (lane >= d) inc += o;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int32_t woff = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) {
        if (w < wid) woff += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return woff + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tile(const int32_t *in, int32_t *out, int64_t n,
                                                            int32_t *bsum) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int32_t v[kScanPer];
    int32_t s = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        v[q] = (base + q < n) ? in[base + q] : 0;
        s += v[q];
    }
    int32_t tot;
    int32_t run = block_exclusive_scan(s, &tot);
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        if (base + q < n) out[base + q] = run;
        run += v[q];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void k_scan_add(int32_t *out, int64_t n, const int32_t *boff, int32_t nb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += boff[i / kScanTile];
    if (i == 0) out[n] = boff[nb];
}

}  // namespace

void scan_exclusive(const int32_t *in, int32_t *out, int64_t n, hipStream_t st) {
    if (n <= 0) {
        HIPCHK(hipMemsetAsync(out, 0, sizeof(int32_t), st));
        return;
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        // one tile: its total is the grand total, written straight to out[n]
        hipLaunchKernelGGL(k_scan_tile, dim3(1), dim3(kScanThreads), 0, st, in, out, n, out + n);
        LAUNCHCHK();
        return;
    }
    DArr<int32_t> bsum(nb + 1);
    hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, out, n, bsum.get());
    LAUNCHCHK();
    scan_exclusive(bsum.get(), bsum.get(), nb, st);   // bsum[0..nb], bsum[nb] = total
    hipLaunchKernelGGL(k_scan_add, dim3(cdiv(n, 256)), dim3(256), 0, st, out, n, bsum.get(), (int32_t)nb);
    LAUNCHCHK();
}

// Device scalars come back through a few pinned host words (one set per host
// thread, kept for the life of the process), so several reads share one
// stream synchronisation.
int32_t *pinned_words() {
    thread_local int32_t *p = nullptr;
    if (!p) HIPCHK(hipHostMalloc(reinterpret_cast<void **>(&p), kPinnedWords * sizeof(int32_t), hipHostMallocDefault));
    return p;
}

void read_ints(std::initializer_list<const int32_t *> src, int32_t *out, hipStream_t st) {
    if (src.size() > (size_t)kPinnedWords) cbs_throw(CBS_ERR_ARG, "too many device scalars in one read");
    int32_t *w = pinned_words();
    int k = 0;
    for (const int32_t *p : src) HIPCHK(hipMemcpyAsync(w + k++, p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < k; ++i) out[i] = w[i];
}

void read_array(const int32_t *dptr, int32_t count, int32_t *out, hipStream_t st) {
    if (count > kPinnedWords) cbs_throw(CBS_ERR_ARG, "too many device scalars in one read");
    int32_t *w = pinned_words();
    if (count > 0) HIPCHK(hipMemcpyAsync(w, dptr, sizeof(int32_t) * count, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < count; ++i) out[i] = w[i];
}

int32_t read_int(const int32_t *dptr, hipStream_t st) {
    int32_t v = 0;
    read_ints({dptr}, &v, st);
    return v;
}

// ------------------------------------------------------------------ pattern
namespace {

// Local face addresses -> global cell ids; flag bad faces.
__global__ void k_globalize(int32_t F, int32_t n_sys, const int64_t *cell_off, const int64_t *face_off,
                            const int32_t *la_in, const int32_t *ua_in, int32_t *la, int32_t *ua,
                            int32_t *flag) {
    const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    int lo = 0, hi = n_sys - 1;            // system s with face_off[s] <= f < face_off[s+1]
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (face_off[mid] <= f) lo = mid; else hi = mid - 1;
    }
    const int64_t c0 = cell_off[lo], nc = cell_off[lo + 1] - c0;
    const int32_t l = la_in[f], u = ua_in[f];
    if (l < 0 || l >= nc || u < 0 || u >= nc || l == u) {
        atomicOr(flag, 1);
        la[f] = 0; ua[f] = 0;
        return;
    }
    la[f] = (int32_t)(c0 + l);
    ua[f] = (int32_t)(c0 + u);
}

__global__ void k_fill_int(int32_t *a, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void k_count(int32_t F, const int32_t *la, const int32_t *ua, int32_t *deg) {
    const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    atomicAdd(&deg[la[f]], 1);
    atomicAdd(&deg[ua[f]], 1);
}

__global__ void k_place_diag(int32_t N, const int32_t *rp, int32_t *col, int32_t *src, int32_t *fill) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    col[rp[i]] = i;
    src[rp[i]] = i;
    fill[i] = rp[i] + 1;
}

// source code: i < N diag; N + f upper face f; N + F + f lower face f
__global__ void k_place_faces(int32_t N, int32_t F, const int32_t *la, const int32_t *ua, int32_t *col,
                              int32_t *src, int32_t *fill) {
    const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const int32_t l = la[f], u = ua[f];
    int32_t p = atomicAdd(&fill[l], 1);
    col[p] = u;
    src[p] = N + f;
    p = atomicAdd(&fill[u], 1);
    col[p] = l;
    src[p] = N + F + f;
}

// Insertion-sort each row by column (makes the atomic placement order
// irrelevant: columns are unique, so the result is deterministic) and flag
// duplicate columns.
__global__ void k_sort_rows(int32_t N, const int32_t *rp, int32_t *col, int32_t *src, int32_t *flag) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t b = rp[i], e = rp[i + 1];
    for (int32_t a = b + 1; a < e; ++a) {
        const int32_t c = col[a], s = src[a];
        int32_t q = a - 1;
        while (q >= b && col[q] > c) {
            col[q + 1] = col[q];
            src[q + 1] = src[q];
            --q;
        }
        col[q + 1] = c;
        src[q + 1] = s;
    }
    for (int32_t a = b + 1; a < e; ++a)
        if (col[a] == col[a - 1]) atomicOr(flag, 2);
}

__global__ void k_slots(int64_t nnzb, int32_t N, int32_t F, const int32_t *src, int32_t *dslot,
                        int32_t *uslot, int32_t *lslot) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnzb) return;
    const int32_t s = src[k];
    if (s < N) dslot[s] = (int32_t)k;
    else if (s < N + F) uslot[s - N] = (int32_t)k;
    else lslot[s - N - F] = (int32_t)k;
}

__global__ void k_mirror(int64_t nnzb, int32_t N, int32_t F, const int32_t *src, const int32_t *uslot,
                         const int32_t *lslot, int32_t *mirror) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnzb) return;
    const int32_t s = src[k];
    if (s < N) mirror[k] = (int32_t)k;
    else if (s < N + F) mirror[k] = lslot[s - N];
    else mirror[k] = uslot[s - N - F];
}

// row id of every system's rows
__global__ void k_row_sys(int32_t N, int32_t n_sys, const int64_t *cell_off, int32_t *row_sys) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int lo = 0, hi = n_sys - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (cell_off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    row_sys[i] = lo;
}

// ------------------------------------------------------------------ values
// One thread per scalar of the block-CSR value array: contiguous writes,
// block-contiguous reads.  Non-finite inputs raise flag bit 4.
// Odd block sizes: one thread per row of a destination block (n contiguous
// values read from the source block, n written to the slot).  Measured on
// MI355X for n = 5 against one thread per value: 0.64 -> 0.61 ms at 1M cells,
// 5.8 -> 4.8 ms at 8M.  Writing in source order instead (contiguous reads,
// each 200-byte block stored at its slot) halved the bandwidth: blocks that
// do not fill whole cache lines are cheap to gather but not to scatter.
template <int n>
__global__ void k_values_rows(int64_t nrows, int32_t N, int32_t F, const int32_t *src, const double *diag,
                              const double *upper, const double *lower, double *vals, int32_t *flag) {
    constexpr int nn = n * n;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nrows) return;
    const int64_t k = g / n;
    const int r = (int)(g - k * n);
    const int32_t s = src[k];
    const double *from = (s < N ? diag + (int64_t)s * nn
                          : (s < N + F ? upper + (int64_t)(s - N) * nn : lower + (int64_t)(s - N - F) * nn)) + r * n;
    double v[n];
#pragma unroll
    for (int c = 0; c < n; ++c) v[c] = from[c];
    bool bad = false;
#pragma unroll
    for (int c = 0; c < n; ++c) {
        bad = bad || !isfinite(v[c]);
        vals[k * nn + r * n + c] = v[c];
    }
    if (bad) atomicOr(flag, 4);
}

template <int n>
__global__ void k_values(int64_t total, int32_t N, int32_t F, const int32_t *src, const double *diag,
                         const double *upper, const double *lower, double *vals, int32_t *flag) {
    // V values per thread (32- or 16-byte accesses when the block size allows)
    constexpr int nn = n * n, V = nn % 4 == 0 ? 4 : (nn % 2 == 0 ? 2 : 1);
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total / V) return;
    const int64_t k = g / (nn / V);
    const int e = (int)(g - k * (nn / V)) * V;
    const int32_t s = src[k];
    const double *from = s < N ? diag + (int64_t)s * nn
                       : (s < N + F ? upper + (int64_t)(s - N) * nn : lower + (int64_t)(s - N - F) * nn);
    double v[V];
    if constexpr (V == 4) {
        typedef double d4 __attribute__((ext_vector_type(4)));
        const d4 a = *reinterpret_cast<const d4 *>(from + e);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    } else if constexpr (V == 2) {
        typedef double d2 __attribute__((ext_vector_type(2)));
        const d2 a = *reinterpret_cast<const d2 *>(from + e);
        v[0] = a.x; v[1] = a.y;
    } else {
        v[0] = from[e];
    }
    bool bad = false;
#pragma unroll
    for (int u = 0; u < V; ++u) {
        bad = bad || !isfinite(v[u]);
        vals[k * nn + e + u] = v[u];
    }
    if (bad) atomicOr(flag, 4);
}

// ------------------------------------------------------------------ assembly
// Per cell, once: u, v, w, the total enthalpy H = (rho E + p)/rho and
// phi = (gamma-1)|u|^2/2, from the conservative state Q = (rho, rho u,
// rho v, rho w, rho E) of an ideal gas with p = (gamma-1)(rho E - rho|u|^2/2).
// Per-cell primitives (u, v, w, H, phi).  A state whose density or pressure
// is not positive (or not a number) sets bit 8 of flag: the Roe average and
// the speed of sound are undefined there even when every coefficient that
// comes out happens to be finite.
__global__ void k_cell_prims(int32_t N, const double *Q, double g, double *prim, int32_t *flag) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double *q = Q + (int64_t)i * 5;
    const double rho = q[0], u = q[1] / rho, v = q[2] / rho, w = q[3] / rho;
    const double g1 = g - 1.0, q2 = u * u + v * v + w * w;
    const double p = g1 * (q[4] - 0.5 * rho * q2);
    if (!(rho > 0.0) || !(p > 0.0)) atomicOr(flag, 8);
    double *o = prim + (int64_t)i * 5;
    o[0] = u; o[1] = v; o[2] = w; o[3] = (q[4] + p) / rho; o[4] = 0.5 * g1 * q2;
}

// Row r of the Euler convective flux Jacobian d(F(Q) . s)/dQ in the
// conservative variables, from the cell's (u, v, w, H, phi); s is an area
// vector and the Jacobian is linear in it.
__device__ inline void euler_jac_row(const double *pr, double sx, double sy, double sz, double g, int r,
                                     double out[5]) {
    const double u = pr[0], v = pr[1], w = pr[2], H = pr[3], phi = pr[4], g1 = g - 1.0;
    const double V = u * sx + v * sy + w * sz;
    if (r == 0) {
        out[0] = 0.0; out[1] = sx; out[2] = sy; out[3] = sz; out[4] = 0.0;
    } else if (r < 4) {
        const double uk = r == 1 ? u : (r == 2 ? v : w), sk = r == 1 ? sx : (r == 2 ? sy : sz);
        out[0] = phi * sk - uk * V;
        out[1] = uk * sx - g1 * u * sk + (r == 1 ? V : 0.0);
        out[2] = uk * sy - g1 * v * sk + (r == 2 ? V : 0.0);
        out[3] = uk * sz - g1 * w * sk + (r == 3 ? V : 0.0);
        out[4] = g1 * sk;
    } else {
        out[0] = V * (phi - H);
        out[1] = H * sx - g1 * u * V;
        out[2] = H * sy - g1 * v * V;
        out[3] = H * sz - g1 * w * V;
        out[4] = g * V;
    }
}

// S lambda of every face, once (the slot kernel reads each face up to 20
// times): the convective spectral radius of the Roe-averaged state,
// |u~ . s| + c~ |s| (weights sqrt(rho), c~^2 = (gamma-1)(H~ - |u~|^2/2)),
// plus |s| times the viscous radius per unit area.
__global__ void k_face_radius(int32_t F, const int32_t *la, const int32_t *ua, const double *Q, const double *prim,
                              const double *Sf, const double *lamv, double g, double *lam) {
    const int32_t f = (int32_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const int32_t l = la[f], r = ua[f];
    const double *pl = prim + (int64_t)l * 5, *pr = prim + (int64_t)r * 5, *s = Sf + (int64_t)f * 3;
    const double al = sqrt(Q[(int64_t)l * 5]), ar = sqrt(Q[(int64_t)r * 5]), wsum = al + ar;
    const double u = (al * pl[0] + ar * pr[0]) / wsum, v = (al * pl[1] + ar * pr[1]) / wsum;
    const double w = (al * pl[2] + ar * pr[2]) / wsum, H = (al * pl[3] + ar * pr[3]) / wsum;
    const double c = sqrt((g - 1.0) * (H - 0.5 * (u * u + v * v + w * w)));
    const double S = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    lam[f] = fabs(u * s[0] + v * s[1] + w * s[2]) + c * S + (lamv ? lamv[f] : 0.0) * S;
}

// The density-based coupled matrix V/dtau I - dR/dQ with the approximate
// Jacobian, written straight into block CSR: one thread per (slot, block
// row r), five values each.  An upper slot (row = owner l, column = u) is
// (J(Q_u, s) - S lambda I)/2, a lower slot (row = u, column = l) is
// (J(Q_l, -s) - S lambda I)/2, and the diagonal of cell i is
// v_dt_i I + (J(Q_i, sum of its outward face vectors) + sum of its S lambda I)/2
// (J is linear in s, so the faces' Jacobians at Q_i add up to one).
// Per cell, once: the sum of its outward face vectors (a face counts +S_f in
// its owner's row and -S_f in its neighbour's) and the sum of its faces'
// S lambda, in the row's slot order.
__global__ void k_cell_faces(int32_t N, int32_t F, const int32_t *rp, const int32_t *src, const double *Sf,
                             const double *lam, double *acc) {
    const int32_t i = (int32_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double nx = 0.0, ny = 0.0, nz = 0.0, lsum = 0.0;
    for (int32_t k2 = rp[i]; k2 < rp[i + 1]; ++k2) {
        const int32_t s2 = src[k2];
        if (s2 < N) continue;
        const bool up = s2 < N + F;
        const int32_t f = up ? s2 - N : s2 - N - F;
        const double *sf = Sf + (int64_t)f * 3;
        const double sg = up ? 1.0 : -1.0;
        nx += sg * sf[0]; ny += sg * sf[1]; nz += sg * sf[2];
        lsum += lam[f];
    }
    double *o = acc + (int64_t)i * 4;
    o[0] = nx; o[1] = ny; o[2] = nz; o[3] = lsum;
}

// One thread per block slot: it gathers the slot's column cell primitives
// and its face (or cell) data once and writes the block's 25 values, row by
// row, into LDS; the workgroup's blocks are one contiguous run of the
// values, stored with unit stride.
constexpr int kAsmSlots = 128;           // block slots per workgroup of the two slot kernels
// The block's column cell (the upper slot's neighbour, the lower slot's owner,
// the diagonal's own cell) is read from the column array, so its primitives
// load in parallel with the face data instead of after the face addresses.
__global__ __launch_bounds__(kAsmSlots) void k_assemble_luo(int64_t nnzb, int32_t N, int32_t F,
                                                            const int32_t *src, const int32_t *col,
                                                            const double *prim,
                                                            const double *Sf, const double *lam,
                                                            const double *cacc, const double *vdt, double g,
                                                            double *vals, int32_t *flag) {
    __shared__ double stage[kAsmSlots * 25];
    const int64_t k0 = (int64_t)blockIdx.x * kAsmSlots;
    const int64_t k = k0 + threadIdx.x;
    const bool act = k < nnzb;
    const int32_t s = act ? src[k] : 0;
    const int32_t j = act ? col[k] : 0;
    const bool face = act && s >= N;
    double pr[5], sv[3], lf, dt;
    const double *p = prim + (int64_t)j * 5;
#pragma unroll
    for (int c = 0; c < 5; ++c) pr[c] = act ? p[c] : 0.0;
    if (face) {
        const bool up = s < N + F;
        const int32_t f = up ? s - N : s - N - F;
        const double sg = up ? 1.0 : -1.0;
        const double *sf = Sf + (int64_t)f * 3;
        sv[0] = sg * sf[0]; sv[1] = sg * sf[1]; sv[2] = sg * sf[2];
        lf = lam[f];
        dt = 0.0;
    } else {
        const double *a = cacc + (int64_t)(act ? s : 0) * 4;
        sv[0] = act ? a[0] : 0.0; sv[1] = act ? a[1] : 0.0; sv[2] = act ? a[2] : 0.0;
        lf = act ? a[3] : 0.0;
        dt = (act && vdt) ? vdt[s] : 0.0;
    }
    bool bad = false;
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        double out[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (act) {
            euler_jac_row(pr, sv[0], sv[1], sv[2], g, r, out);
            if (face) {
#pragma unroll
                for (int c = 0; c < 5; ++c) out[c] = 0.5 * (out[c] - (c == r ? lf : 0.0));
            } else {
#pragma unroll
                for (int c = 0; c < 5; ++c) out[c] = 0.5 * (out[c] + (c == r ? lf : 0.0)) + (c == r ? dt : 0.0);
            }
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            bad = bad || !isfinite(out[c]);
            stage[threadIdx.x * 25 + r * 5 + c] = out[c];
        }
    }
    if (bad) atomicOr(flag, 4);
    __syncthreads();
    const int64_t total = nnzb * 25, base = k0 * 25;
#pragma unroll
    for (int q = 0; q < 25; ++q) {
        const int64_t e = base + threadIdx.x + q * kAsmSlots;
        if (e < total) vals[e] = stage[threadIdx.x + q * kAsmSlots];
    }
}

// ---------------------------------------------- pressure-based (p, U) blocks
// Seen from row i, face f (slot code s) has area vector sg S_f, volume flux
// sg F_f and the row's own interpolation weight w = f_x (owner) or 1 - f_x.
// Per cell: the momentum diagonal a_ii^uu = uu_add + sum of (max(sg F, 0) + k_f)
// with the diffusion k_f = nu |S| / (n . d), D_i = V_i / a_ii^uu, and the
// up/pu diagonal vector sum of w sg S_f.
__global__ void k_pu_cells(int32_t N, int32_t F, const int32_t *rp, const int32_t *src, const double *Sf,
                           const double *fx, const double *dv, const double *flux, const double *nu,
                           const double *vol, const double *uu_add, double *acc) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double auu = uu_add ? uu_add[i] : 0.0, ux = 0.0, uy = 0.0, uz = 0.0;
    for (int32_t k2 = rp[i]; k2 < rp[i + 1]; ++k2) {
        const int32_t s2 = src[k2];
        if (s2 < N) continue;
        const bool up = s2 < N + F;
        const int32_t f = up ? s2 - N : s2 - N - F;
        const double *S = Sf + (int64_t)f * 3, *d = dv + (int64_t)f * 3;
        const double Sm = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
        const double nd = (S[0] * d[0] + S[1] * d[1] + S[2] * d[2]) / Sm;
        const double sg = up ? 1.0 : -1.0, w = up ? fx[f] : 1.0 - fx[f];
        auu += fmax(sg * flux[f], 0.0) + nu[f] * Sm / nd;
        ux += w * sg * S[0]; uy += w * sg * S[1]; uz += w * sg * S[2];
    }
    double *o = acc + (int64_t)i * 5;
    o[0] = auu; o[1] = vol[i] / auu; o[2] = ux; o[3] = uy; o[4] = uz;
}

// Per face: the Rhie-Chow coefficient (f_x D_l + (1 - f_x) D_u) |S| / (n . d)
// and the diffusion coefficient k_f.
__global__ void k_pu_faces(int32_t F, const int32_t *la, const int32_t *ua, const double *Sf, const double *fx,
                           const double *dv, const double *nu, const double *acc, double *fc) {
    const int32_t f = (int32_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const double *S = Sf + (int64_t)f * 3, *d = dv + (int64_t)f * 3;
    const double Sm = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
    const double nd = (S[0] * d[0] + S[1] * d[1] + S[2] * d[2]) / Sm;
    const double Df = fx[f] * acc[(int64_t)la[f] * 5 + 1] + (1.0 - fx[f]) * acc[(int64_t)ua[f] * 5 + 1];
    fc[2 * (int64_t)f] = Df * Sm / nd;
    fc[2 * (int64_t)f + 1] = nu[f] * Sm / nd;
}

// Per cell: the pp diagonal, pp_add plus the row's Rhie-Chow coefficients.
__global__ void k_pu_pp(int32_t N, int32_t F, const int32_t *rp, const int32_t *src, const double *fc,
                        const double *pp_add, double *pp) {
    const int32_t i = (int32_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double a = pp_add ? pp_add[i] : 0.0;
    for (int32_t k2 = rp[i]; k2 < rp[i + 1]; ++k2) {
        const int32_t s2 = src[k2];
        if (s2 < N) continue;
        a += fc[2 * (int64_t)(s2 < N + F ? s2 - N : s2 - N - F)];
    }
    pp[i] = a;
}

// One thread per block slot, its 16 values staged in LDS like the
// density-based kernel.  Row 0 is continuity (pp, pu), rows 1-3 momentum
// (up, uu = scalar times I).
__global__ __launch_bounds__(kAsmSlots) void k_assemble_pu(int64_t nnzb, int32_t N, int32_t F, const int32_t *src,
                                                           const double *Sf, const double *fx, const double *flux,
                                                           const double *fc, const double *acc, const double *pp,
                                                           double *vals, int32_t *flag) {
    // one thread per block slot, its 16 values staged in LDS as in
    // k_assemble_luo
    __shared__ double stage[kAsmSlots * 16];
    const int64_t k0 = (int64_t)blockIdx.x * kAsmSlots;
    const int64_t k = k0 + threadIdx.x;
    const bool act = k < nnzb;
    const int32_t s = act ? src[k] : 0;
    double out[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) out[e] = 0.0;
    if (act && s >= N) {
        const bool up = s < N + F;
        const int32_t f = up ? s - N : s - N - F;
        const double sg = up ? 1.0 : -1.0, w = up ? fx[f] : 1.0 - fx[f];
        const double *S = Sf + (int64_t)f * 3;
        const double cpl = (1.0 - w) * sg;              // coupling vector (1 - w) sg S
        const double c0 = cpl * S[0], c1 = cpl * S[1], c2 = cpl * S[2];
        const double uu = -(fmax(-sg * flux[f], 0.0) + fc[2 * (int64_t)f + 1]);
        out[0] = -fc[2 * (int64_t)f];
        out[1] = c0; out[2] = c1; out[3] = c2;
        out[4] = c0; out[5] = uu;
        out[8] = c1; out[10] = uu;
        out[12] = c2; out[15] = uu;
    } else if (act) {
        const double *a = acc + (int64_t)s * 5;
        const double a0 = a[0], a2 = a[2], a3 = a[3], a4 = a[4];
        out[0] = pp[s];
        out[1] = a2; out[2] = a3; out[3] = a4;
        out[4] = a2; out[5] = a0;
        out[8] = a3; out[10] = a0;
        out[12] = a4; out[15] = a0;
    }
    bool bad = false;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        bad = bad || !isfinite(out[e]);
        stage[threadIdx.x * 16 + e] = out[e];
    }
    if (bad) atomicOr(flag, 4);
    __syncthreads();
    const int64_t total = nnzb * 16, base = k0 * 16;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int64_t e = base + threadIdx.x + q * kAsmSlots;
        if (e < total) vals[e] = stage[threadIdx.x + q * kAsmSlots];
    }
}

__global__ void k_check_finite(const double *a, int64_t count, int32_t *flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count && !isfinite(a[i])) atomicOr(flag, 4);
}

}  // namespace

void convert_pattern(cbs_system *h) {
    hipStream_t st = h->stream;
    const int32_t N = h->N, F = h->F;
    DArr<int32_t> deg(N + 1);
    hipLaunchKernelGGL(k_fill_int, dim3(cdiv(N, 256)), dim3(256), 0, st, deg.get(), (int64_t)N, 1);
    if (F > 0)
        hipLaunchKernelGGL(k_count, dim3(cdiv(F, 256)), dim3(256), 0, st, F, h->la.get(), h->ua.get(), deg.get());
    LAUNCHCHK();
    h->rp.alloc(N + 1);
    scan_exclusive(deg.get(), h->rp.get(), N, st);
    h->nnzb = (int64_t)N + 2 * (int64_t)F;
    const int64_t nnzb = h->nnzb;
    h->col.alloc(nnzb);
    h->src.alloc(nnzb);
    hipLaunchKernelGGL(k_place_diag, dim3(cdiv(N, 256)), dim3(256), 0, st, N, h->rp.get(), h->col.get(),
                       h->src.get(), deg.get());
    if (F > 0)
        hipLaunchKernelGGL(k_place_faces, dim3(cdiv(F, 256)), dim3(256), 0, st, N, F, h->la.get(), h->ua.get(),
                           h->col.get(), h->src.get(), deg.get());
    HIPCHK(hipMemsetAsync(h->dflag.get(), 0, sizeof(int32_t), st));
    hipLaunchKernelGGL(k_sort_rows, dim3(cdiv(N, 256)), dim3(256), 0, st, N, h->rp.get(), h->col.get(),
                       h->src.get(), h->dflag.get());
    LAUNCHCHK();
    if (read_int(h->dflag.get(), st) != 0) cbs_throw(CBS_ERR_PATTERN, "duplicate face (same cell pair twice)");
    h->dslot.alloc(N);
    h->uslot.alloc(F > 0 ? F : 1);
    h->lslot.alloc(F > 0 ? F : 1);
    h->mirror.alloc(nnzb);
    hipLaunchKernelGGL(k_slots, dim3(cdiv(nnzb, 256)), dim3(256), 0, st, nnzb, N, F, h->src.get(),
                       h->dslot.get(), h->uslot.get(), h->lslot.get());
    hipLaunchKernelGGL(k_mirror, dim3(cdiv(nnzb, 256)), dim3(256), 0, st, nnzb, N, F, h->src.get(),
                       h->uslot.get(), h->lslot.get(), h->mirror.get());
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(st));
}

// exposed for the batched create
void globalize_faces(cbs_system *h, const int32_t *la_in, const int32_t *ua_in) {
    hipStream_t st = h->stream;
    const int32_t F = h->F;
    DArr<int64_t> coff(h->n_sys + 1), foff(h->n_sys + 1);
    HIPCHK(hipMemcpyAsync(coff.get(), h->cell_off.data(), sizeof(int64_t) * (h->n_sys + 1),
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(foff.get(), h->face_off.data(), sizeof(int64_t) * (h->n_sys + 1),
                          hipMemcpyHostToDevice, st));
    h->la.alloc(F > 0 ? F : 1);
    h->ua.alloc(F > 0 ? F : 1);
    HIPCHK(hipMemsetAsync(h->dflag.get(), 0, sizeof(int32_t), st));
    if (F > 0)
        hipLaunchKernelGGL(k_globalize, dim3(cdiv(F, 256)), dim3(256), 0, st, F, h->n_sys, coff.get(), foff.get(),
                           la_in, ua_in, h->la.get(), h->ua.get(), h->dflag.get());
    LAUNCHCHK();
    if (read_int(h->dflag.get(), st) != 0)
        cbs_throw(CBS_ERR_PATTERN, "face index out of range or self face (lower_addr == upper_addr)");
    // per-row system ids of level 0 are built in amg setup from cell_off
    HIPCHK(hipStreamSynchronize(st));
}

void build_row_sys(cbs_system *h, Level &L0) {
    DArr<int64_t> coff(h->n_sys + 1);
    HIPCHK(hipMemcpyAsync(coff.get(), h->cell_off.data(), sizeof(int64_t) * (h->n_sys + 1),
                          hipMemcpyHostToDevice, h->stream));
    L0.row_sys.alloc(h->N);
    hipLaunchKernelGGL(k_row_sys, dim3(cdiv(h->N, 256)), dim3(256), 0, h->stream, h->N, h->n_sys, coff.get(),
                       L0.row_sys.get());
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(h->stream));
}

void convert_values(cbs_system *h, const double *diag, const double *upper, const double *lower) {
    hipStream_t st = h->stream;
    const int n = h->n;
    const int64_t total = h->nnzb * n * n;
    h->vals.ensure(total);
    HIPCHK(hipMemsetAsync(h->dflag.get(), 0, sizeof(int32_t), st));
    const dim3 b(256);
    const int32_t *sp = h->src.get();
    double *vp = h->vals.get();
    int32_t *fp = h->dflag.get();
    if (n % 2 == 1 && n > 1) {
        const int64_t nr = h->nnzb * n;
        const dim3 g(cdiv(nr, 256));
        if (n == 3) hipLaunchKernelGGL(k_values_rows<3>, g, b, 0, st, nr, h->N, h->F, sp, diag, upper, lower, vp, fp);
        else hipLaunchKernelGGL(k_values_rows<5>, g, b, 0, st, nr, h->N, h->F, sp, diag, upper, lower, vp, fp);
    } else {
        const int64_t nthr = (n * n) % 4 == 0 ? total / 4 : ((n * n) % 2 == 0 ? total / 2 : total);
        const dim3 g(cdiv(nthr, 256));
        switch (n) {
            case 1: hipLaunchKernelGGL(k_values<1>, g, b, 0, st, total, h->N, h->F, sp, diag, upper, lower, vp, fp); break;
            case 2: hipLaunchKernelGGL(k_values<2>, g, b, 0, st, total, h->N, h->F, sp, diag, upper, lower, vp, fp); break;
            case 4: hipLaunchKernelGGL(k_values<4>, g, b, 0, st, total, h->N, h->F, sp, diag, upper, lower, vp, fp); break;
            default: cbs_throw(CBS_ERR_ARG, "bdim must be 1..5");
        }
    }
    LAUNCHCHK();
    if (read_int(h->dflag.get(), st) & 4) cbs_throw(CBS_ERR_NONFINITE, "non-finite matrix coefficient");
}

// The four density-based assembly passes on caller-supplied scratch:
// face_lam[F], prim[5N], acc[4N] (each fully written before it is read) and
// an int32 flag that must be zero on entry.
static void assemble_luo_on(cbs_system *h, const double *Q, const double *Sf, const double *lam_visc,
                            const double *v_dt, double gamma, double *face_lam, double *prim, double *acc,
                            int32_t *flag) {
    hipStream_t st = h->stream;
    hipLaunchKernelGGL(k_cell_prims, dim3(cdiv(h->N, 256)), dim3(256), 0, st, h->N, Q, gamma, prim, flag);
    if (h->F > 0)
        hipLaunchKernelGGL(k_face_radius, dim3(cdiv(h->F, 256)), dim3(256), 0, st, h->F, h->la.get(), h->ua.get(), Q,
                           prim, Sf, lam_visc, gamma, face_lam);
    hipLaunchKernelGGL(k_cell_faces, dim3(cdiv(h->N, 256)), dim3(256), 0, st, h->N, h->F, h->rp.get(), h->src.get(),
                       Sf, face_lam, acc);
    const int64_t nthr = h->nnzb * 5;
    if (nthr > 0)
        hipLaunchKernelGGL(k_assemble_luo, dim3(cdiv(h->nnzb, kAsmSlots)), dim3(kAsmSlots), 0, st, h->nnzb, h->N,
                           h->F,
                           h->src.get(), h->col.get(), prim, Sf, face_lam, acc, v_dt, gamma, h->vals.get(), flag);
    LAUNCHCHK();
}

static void luo_flag_errors(int32_t fl) {
    if (fl & 8) cbs_throw(CBS_ERR_NONFINITE, "a cell state with non-positive density or pressure");
    if (fl & 4) cbs_throw(CBS_ERR_NONFINITE, "non-finite assembled coefficient");
}

void assemble_luo(cbs_system *h, const double *Q, const double *Sf, const double *lam_visc, const double *v_dt,
                  double gamma) {
    hipStream_t st = h->stream;
    h->vals.ensure((size_t)h->nnzb * 25);
    HIPCHK(hipMemsetAsync(h->dflag.get(), 0, sizeof(int32_t), st));
    h->face_lam.ensure(h->F > 0 ? (size_t)h->F : 1);
    h->cell_prim.ensure((size_t)h->N * 5);
    h->cell_acc.ensure((size_t)h->N * 4);
    assemble_luo_on(h, Q, Sf, lam_visc, v_dt, gamma, h->face_lam.get(), h->cell_prim.get(), h->cell_acc.get(),
                    h->dflag.get());
    luo_flag_errors(read_int(h->dflag.get(), st));
}

// ------------------------------------------- assembly without allocation
// The density-based assembly for callers that cannot allocate device memory:
// its per-face and per-cell passes run on a fixed array that the library
// holds on every device it runs on, for the life of the process.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in symbol); the device address comes from hipGetSymbolAddress, once
// per device, with that device current.
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

double *scratch_on(int dev) {
    if (dev < 0 || dev >= kMaxDevices) cbs_throw(CBS_ERR_HIP, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        HIPCHK(hipGetDevice(&cur));
        if (cur != dev) HIPCHK(hipSetDevice(dev));
        double *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(reinterpret_cast<void **>(&p), HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            cbs_throw(CBS_ERR_HIP, std::string("hipGetSymbolAddress of the assembly scratch failed: ") +
                                       hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

// doubles of each scratch segment, rounded up to 256 bytes
inline size_t seg(size_t count) { return (count + 31) & ~(size_t)31; }
}  // namespace

size_t assemble_luo_scratch_bytes(int64_t N, int64_t F) {
    return (seg(1) + seg((size_t)(F > 0 ? F : 1)) + seg((size_t)N * 5) + seg((size_t)N * 4)) * sizeof(double);
}

void assemble_luo_noalloc(cbs_system *h, const double *Q, const double *Sf, const double *lam_visc,
                          const double *v_dt, double gamma) {
    const size_t need = assemble_luo_scratch_bytes(h->N, h->F);
    if (need > kNoAllocScratchBytes)
        cbs_throw(CBS_ERR_ARG, "the system needs " + std::to_string(need) + " bytes of assembly scratch, more than the " +
                                   std::to_string(kNoAllocScratchBytes) + " the allocation-free assembly holds");
    if (h->vals.n < (size_t)h->nnzb * 25) cbs_throw(CBS_ERR_STATE, "block-CSR values are not allocated");
    hipStream_t st = h->stream;
    double *base = scratch_on(h->device);
    int32_t *flag = reinterpret_cast<int32_t *>(base);
    double *face_lam = base + seg(1);
    double *prim = face_lam + seg((size_t)(h->F > 0 ? h->F : 1));
    double *acc = prim + seg((size_t)h->N * 5);
    // the flag keeps the last call's value: clear it with a kernel
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, flag, (int64_t)1, 0);
    assemble_luo_on(h, Q, Sf, lam_visc, v_dt, gamma, face_lam, prim, acc, flag);
    int32_t fl = 0;
    HIPCHK(hipMemcpyAsync(&fl, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    luo_flag_errors(fl);
}

void assemble_pu(cbs_system *h, const double *Sf, const double *fx, const double *d, const double *flux,
                 const double *nu, const double *vol, const double *uu_add, const double *pp_add) {
    hipStream_t st = h->stream;
    h->vals.ensure((size_t)h->nnzb * 16);
    HIPCHK(hipMemsetAsync(h->dflag.get(), 0, sizeof(int32_t), st));
    h->cell_acc.ensure((size_t)h->N * 5);
    h->cell_prim.ensure((size_t)h->N);
    h->face_lam.ensure(h->F > 0 ? 2 * (size_t)h->F : 1);
    hipLaunchKernelGGL(k_pu_cells, dim3(cdiv(h->N, 256)), dim3(256), 0, st, h->N, h->F, h->rp.get(), h->src.get(), Sf,
                       fx, d, flux, nu, vol, uu_add, h->cell_acc.get());
    if (h->F > 0)
        hipLaunchKernelGGL(k_pu_faces, dim3(cdiv(h->F, 256)), dim3(256), 0, st, h->F, h->la.get(), h->ua.get(), Sf, fx,
                           d, nu, h->cell_acc.get(), h->face_lam.get());
    hipLaunchKernelGGL(k_pu_pp, dim3(cdiv(h->N, 256)), dim3(256), 0, st, h->N, h->F, h->rp.get(), h->src.get(),
                       h->face_lam.get(), pp_add, h->cell_prim.get());
    const int64_t nthr = h->nnzb * 4;
    if (nthr > 0)
        hipLaunchKernelGGL(k_assemble_pu, dim3(cdiv(h->nnzb, kAsmSlots)), dim3(kAsmSlots), 0, st, h->nnzb, h->N, h->F,
                           h->src.get(), Sf, fx, flux, h->face_lam.get(), h->cell_acc.get(), h->cell_prim.get(),
                           h->vals.get(), h->dflag.get());
    LAUNCHCHK();
    if (read_int(h->dflag.get(), st) & 4)
        cbs_throw(CBS_ERR_NONFINITE, "non-finite assembled coefficient (zero momentum diagonal or n . d = 0)");
}

void check_finite(const double *a, int64_t count, int32_t *dflag, hipStream_t st) {
    HIPCHK(hipMemsetAsync(dflag, 0, sizeof(int32_t), st));
    if (count > 0) hipLaunchKernelGGL(k_check_finite, dim3(cdiv(count, 256)), dim3(256), 0, st, a, count, dflag);
    LAUNCHCHK();
    if (read_int(dflag, st) & 4) cbs_throw(CBS_ERR_NONFINITE, "non-finite entry in right-hand side or guess");
}

// ------------------------------------------------------------------ packing
namespace {
__global__ void k_pack(int32_t N, int32_t n, const double *soa, double *aos) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)N * n) return;
    const int64_t i = g / n;
    const int v = (int)(g - i * n);
    aos[g] = soa[(int64_t)v * N + i];
}
__global__ void k_unpack(int32_t N, int32_t n, const double *aos, double *soa) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)N * n) return;
    const int v = (int)(g / N);
    const int64_t i = g - (int64_t)v * N;
    soa[g] = aos[i * n + v];
}

template <int n>
__global__ void k_grad(int32_t N, int32_t F, const int32_t *la, const int32_t *ua, const double *lam,
                       const double *x, double *gd, double *gu, double *gl) {
    constexpr int nn = n * n;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nd = (int64_t)N * nn, nf = (int64_t)F * nn;
    if (g < nd) {
        const int64_t i = g / nn;
        const int e = (int)(g - i * nn), r = e / n, c = e - r * n;
        gd[g] = -lam[i * n + r] * x[i * n + c];
    } else if (g < nd + nf) {
        const int64_t q = g - nd, f = q / nn;
        const int e = (int)(q - f * nn), r = e / n, c = e - r * n;
        const int64_t l = la[f], u = ua[f];
        gu[q] = -lam[l * n + r] * x[u * n + c];
        gl[q] = -lam[u * n + r] * x[l * n + c];
    }
}
}  // namespace

void pack_fields(int32_t N, int32_t n, const double *soa, double *aos, hipStream_t st) {
    const int64_t m = (int64_t)N * n;
    if (m > 0) hipLaunchKernelGGL(k_pack, dim3(cdiv(m, 256)), dim3(256), 0, st, N, n, soa, aos);
    LAUNCHCHK();
}

void unpack_fields(int32_t N, int32_t n, const double *aos, double *soa, hipStream_t st) {
    const int64_t m = (int64_t)N * n;
    if (m > 0) hipLaunchKernelGGL(k_unpack, dim3(cdiv(m, 256)), dim3(256), 0, st, N, n, aos, soa);
    LAUNCHCHK();
}

void gradient(cbs_system *h, const double *lam, const double *x, double *gd, double *gu, double *gl) {
    const int64_t tot = ((int64_t)h->N + h->F) * h->n * h->n;
    const dim3 g(cdiv(tot, 256)), b(256);
    hipStream_t st = h->stream;
    switch (h->n) {
        case 1: hipLaunchKernelGGL(k_grad<1>, g, b, 0, st, h->N, h->F, h->la.get(), h->ua.get(), lam, x, gd, gu, gl); break;
        case 2: hipLaunchKernelGGL(k_grad<2>, g, b, 0, st, h->N, h->F, h->la.get(), h->ua.get(), lam, x, gd, gu, gl); break;
        case 3: hipLaunchKernelGGL(k_grad<3>, g, b, 0, st, h->N, h->F, h->la.get(), h->ua.get(), lam, x, gd, gu, gl); break;
        case 4: hipLaunchKernelGGL(k_grad<4>, g, b, 0, st, h->N, h->F, h->la.get(), h->ua.get(), lam, x, gd, gu, gl); break;
        case 5: hipLaunchKernelGGL(k_grad<5>, g, b, 0, st, h->N, h->F, h->la.get(), h->ua.get(), lam, x, gd, gu, gl); break;
    }
    LAUNCHCHK();
}
