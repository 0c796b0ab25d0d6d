// Kernels and launchers: labelling (Alg. 2 Step 2), explicit pair lists,
// one segment's pairwise matrix, and the cost tiles of Eq. (1).
//
// Pairs are grouped by support class so each runs in the narrowest group
// shape that holds it (rows = the larger support, T; columns, S):
//   class 0: T <= 16            -> 16 lanes, 16 columns, cost rows in registers
//   class 1: 16 < T <= 32       -> 32 lanes, 32 columns, registers
//   class 2: T > 32, S <= 32    -> 64 lanes, 32 columns, registers
//   class 3: T > 32, S > 32     -> 64 lanes, 64 columns, cost tile in LDS
// Objects are counting-sorted by support on the device, which makes every
// class a contiguous range of rows (labelling) or of pair indices (pairwise
// matrix); pairwise classes are drained by persistent workgroups through an
// atomic work counter.  Results do not depend on the schedule: every shape
// computes the same bits, and each pair is oriented by its own indices.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "d2_internal.h"
#include "d2_shapes.h"
#include "d2_solver.h"

namespace d2 {

// Support-value bucket: 0..64, and 65 for anything larger (reported as too
// large by the solver).
__device__ __forceinline__ int support_bucket(const int64_t *off, int64_t i) {
    const int64_t t = off[i + 1] - off[i];
    return t < 0 ? 0 : (t > 64 ? 65 : (int)t);
}

// ------------------------------------------------------ support sorting

// ws layout (all int64): hist[66] | cursor[66] | bounds[8] | counters[32] | perm[n]
// (work-queue counters: one per support class and XCD)
struct SortWS {
    int64_t *hist, *cursor, *bounds;
    unsigned long long *counters;
    int64_t *perm;
};

__device__ __forceinline__ SortWS sort_ws(void *ws) {
    int64_t *p = (int64_t *)ws;
    SortWS s;
    s.hist = p;
    s.cursor = p + 66;
    s.bounds = p + 132;
    s.counters = (unsigned long long *)(p + 140);
    s.perm = p + 172;
    return s;
}

size_t sort_ws_bytes(int64_t n) { return (size_t)(172 + (n > 0 ? n : 0)) * sizeof(int64_t); }

__global__ void k_sort_init(void *ws) {
    SortWS s = sort_ws(ws);
    const int t = threadIdx.x;
    if (t < 66) { s.hist[t] = 0; s.cursor[t] = 0; }
    if (t < 8) s.bounds[t] = 0;
    if (t < 32) s.counters[t] = 0ull;
}

__global__ void k_sort_hist(KSet X, void *ws) {
    SortWS s = sort_ws(ws);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < X.n;
         i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd((unsigned long long *)&s.hist[support_bucket(X.off, i)], 1ull);
}

// Exclusive prefix over buckets, and class boundaries: bounds[c] = number of
// sorted objects whose class is <= c (class is monotone in the support).
// mode 0 (pairwise): class by the support alone (<= e0, <= e1, larger; the
// bin edges e0 <= 16 and e1 <= 32 keep every class within its shape).
// mode 1 (labelling against centroids of support <= smax): class of the
// pair (max(t, smax), min(t, smax)).
__global__ void k_sort_scan(void *ws, int64_t n, int mode, int smax, int e0, int e1) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    SortWS s = sort_ws(ws);
    int64_t acc = 0;
    int64_t le[4] = {0, 0, 0, 0};
    for (int t = 0; t < 66; ++t) {
        s.cursor[t] = acc;
        const int64_t T = t > smax ? t : smax, S = t < smax ? t : smax;
        const int c = mode == 0 ? (t <= e0 ? 0 : (t <= e1 ? 1 : 2)) : class_of(T, S);
        const int64_t h = s.hist[t];
        acc += h;
        for (int k = c; k < 4; ++k) le[k] += h;
    }
    for (int k = 0; k < 4; ++k) s.bounds[k] = le[k];
}

__global__ void k_sort_scatter(KSet X, void *ws) {
    SortWS s = sort_ws(ws);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < X.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int b = support_bucket(X.off, i);
        const int64_t pos = (int64_t)atomicAdd((unsigned long long *)&s.cursor[b], 1ull);
        s.perm[pos] = i;
    }
}

// ---------------------------------------------------------- labelling

// Rows [row_lo, row_hi) of the (optionally permuted) row order, each against
// centroid chunk c of `chunks`; one workgroup per (row, chunk) item.
template <int CLS, typename TIn, int START>
__global__ __launch_bounds__(ShapeCfg<CLS>::threads, ShapeCfg<CLS>::occ) void k_assign(
    KSet X, KSet Z, KOpts o, const int64_t *perm, const int64_t *bounds, int cls_lo_idx,
    int64_t row_begin, int64_t row_end, int64_t chunks, int64_t per_chunk, int32_t *labels,
    double *best, double *all, int32_t *row_status, double *ws_best, int32_t *ws_label,
    int32_t *ws_status) {
    constexpr int G = ShapeCfg<CLS>::G, GS = ShapeCfg<CLS>::GS, NG = ShapeCfg<CLS>::groups;
    constexpr bool LT = ShapeCfg<CLS>::LT;
    __shared__ GroupMem<G, GS> mem[NG];
    __shared__ TileOf<CLS, START> ltile[NG];
    __shared__ double red_v[NG];
    __shared__ int red_i[NG], red_s[NG];
    const int tid = threadIdx.x;
    const int g = tid / G, l = tid % G, gbase = (tid & 63) & ~(G - 1);
    int64_t row_lo = row_begin, row_hi = row_end;
    if (bounds) {
        row_lo = cls_lo_idx > 0 ? bounds[cls_lo_idx - 1] : 0;
        row_hi = bounds[cls_lo_idx];
    }
    const int64_t total = (row_hi - row_lo) * chunks;
    const int64_t K = Z.n;
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int64_t r = row_lo + item / chunks, ch = item % chunks;
        const int64_t i = perm ? perm[r] : r;
        const int64_t j0 = ch * per_chunk;
        const int64_t j1 = j0 + per_chunk < K ? j0 + per_chunk : K;
        double bv = INFINITY;
        int bj = kNoKey, worst = kOk;
        for (int64_t j = j0 + g; j < j1; j += NG) {
            NodeState<G, GS, LT> N;
            PairView pv = orient(X, i, Z, j, (int)sizeof(TIn));
            SolveOut res = solve_pair<G, GS, LT, TIn, START>(mem[g], ltile[g], N, pv, X.d, o, l, gbase);
            if (res.status != kOk) {
                worst = res.status > worst ? res.status : worst;
                res.d2 = __builtin_nan("");
            } else if (res.d2 < bv || (res.d2 == bv && (int)j < bj)) {
                bv = res.d2;
                bj = (int)j;
            }
            if (all && l == 0) all[i * K + j] = res.d2;
        }
        if (l == 0) { red_v[g] = bv; red_i[g] = bj; red_s[g] = worst; }
        __syncthreads();
        if (tid == 0) {
            double v = INFINITY;
            int jj = kNoKey, st = kOk;
            for (int q = 0; q < NG; ++q) {
                if (red_v[q] < v || (red_v[q] == v && red_i[q] < jj)) { v = red_v[q]; jj = red_i[q]; }
                st = red_s[q] > st ? red_s[q] : st;
            }
            if (chunks == 1) {
                labels[i] = st == kOk ? jj : -1;
                best[i] = st == kOk ? v : __builtin_nan("");
                if (row_status) row_status[i] = st;
            } else {
                ws_best[i * chunks + ch] = v;
                ws_label[i * chunks + ch] = jj;
                ws_status[i * chunks + ch] = st;
            }
        }
        __syncthreads();
    }
}

__global__ void k_assign_reduce(int64_t n, int64_t chunks, const double *ws_best,
                                const int32_t *ws_label, const int32_t *ws_status, int32_t *labels,
                                double *best, int32_t *row_status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = INFINITY;
    int jj = kNoKey, st = kOk;
    for (int64_t c = 0; c < chunks; ++c) {
        const double bv = ws_best[i * chunks + c];
        const int bj = ws_label[i * chunks + c];
        if (bv < v || (bv == v && bj < jj)) { v = bv; jj = bj; }
        const int s = ws_status[i * chunks + c];
        st = s > st ? s : st;
    }
    labels[i] = st == kOk ? jj : -1;
    best[i] = st == kOk ? v : __builtin_nan("");
    if (row_status) row_status[i] = st;
}

// ------------------------------------------------------- explicit pairs

template <int CLS, typename TIn, int START>
__global__ __launch_bounds__(ShapeCfg<CLS>::threads, ShapeCfg<CLS>::occ) void k_emd_pairs(
    KSet A, KSet B, const int64_t *pairs, int64_t npairs, KOpts o, double *dist,
    const int64_t *plan_off, double *plan, const int64_t *dual_off, double *duals, int32_t *status,
    int32_t *pivots) {
    constexpr int G = ShapeCfg<CLS>::G, GS = ShapeCfg<CLS>::GS, NG = ShapeCfg<CLS>::groups;
    constexpr bool LT = ShapeCfg<CLS>::LT;
    __shared__ GroupMem<G, GS> mem[NG];
    __shared__ TileOf<CLS, START> tiles[NG];
    const int tid = threadIdx.x;
    const int g = tid / G, l = tid % G, gbase = (tid & 63) & ~(G - 1);
    const int64_t stride = (int64_t)gridDim.x * NG;
    for (int64_t k = (int64_t)blockIdx.x * NG + g; k < npairs; k += stride) {
        const int64_t i = pairs[2 * k], j = pairs[2 * k + 1];
        int st, npiv = 0, nbland = 0;
        double val = __builtin_nan("");
        if (i < 0 || i >= A.n || j < 0 || j >= B.n) {
            st = kTooLarge;
        } else {
            NodeState<G, GS, LT> N;
            PairView pv = orient(A, i, B, j, (int)sizeof(TIn));
            SolveOut r = solve_pair<G, GS, LT, TIn, START>(mem[g], tiles[g], N, pv, A.d, o, l, gbase);
            st = r.status;
            npiv = r.pivots;
            nbland = r.bland_pivots;
            if (st == kOk) {
                val = r.d2;
                if (plan || duals)
                    write_certificate<G, GS, LT>(mem[g], N, pv, l, plan ? plan + plan_off[k] : nullptr,
                                                 duals ? duals + dual_off[k] : nullptr);
            }
        }
        if (l == 0) {
            dist[k] = val;
            if (status) status[k] = st;
            if (pivots) { pivots[2 * k] = npiv; pivots[2 * k + 1] = nbland; }
        }
    }
}

// ------------------------------------------------------------ pairwise

// Position of pair (i, j), i < j, in the condensed row-major order.
__device__ __forceinline__ int64_t condensed_index(int64_t n, int64_t i, int64_t j) {
    return i * n - i * (i + 1) / 2 + (j - i - 1);
}

// The pairs of one support class, in sorted-object positions: every (a, b)
// with a in [A0, A1), b in [B0, B1) and a < b.
//   class 0: both in [0, n16); class 1: b in [n16, n32), any a < b;
//   class 2: a in [0, n32), b in [n32, n); class 3: both in [n32, n).
struct Region {
    int64_t A0, A1, B0, B1;
};

__device__ __forceinline__ Region class_region(int cls, int64_t n16, int64_t n32, int64_t n) {
    switch (cls) {
    case 0: return Region{0, n16, 0, n16};
    case 1: return Region{0, n32, n16, n32};
    case 2: return Region{0, n32, n32, n};
    default: return Region{n32, n, n32, n};
    }
}

// Items are walked tile by tile: a tile holds `ta` consecutive a positions
// (at most 64 tiles per class), and within a tile b runs outermost, so
// consecutive items share their b object and a tile's a objects are reused
// while it is worked on.  Pairs of tile [a0, a1): for b from
// bs = max(B0, a0 + 1) on, the a in [a0, min(a1, b)).
__device__ __forceinline__ int64_t tile_width(const Region &R, int tile) {
    const int64_t span = R.A1 - R.A0;
    const int64_t min_w = (span + 63) / 64;
    const int64_t w = tile > 0 ? tile : 128;
    return w > min_w ? w : (min_w > 0 ? min_w : 1);
}

__device__ __forceinline__ int64_t tri2(int64_t m) { return m > 1 ? m * (m - 1) / 2 : 0; }

__device__ __forceinline__ void tile_counts(const Region &R, int64_t a0, int64_t a1, int64_t &c1, int64_t &c2) {
    const int64_t bs = R.B0 > a0 + 1 ? R.B0 : a0 + 1;
    const int64_t e1 = a1 < R.B1 ? a1 : R.B1;
    c1 = e1 > bs ? tri2(e1 - a0) - tri2(bs - a0) : 0;   // b < a1: b - a0 pairs each
    const int64_t b2 = bs > a1 ? bs : a1;
    c2 = R.B1 > b2 ? (R.B1 - b2) * (a1 - a0) : 0;        // b >= a1: the whole tile each
}

__device__ __forceinline__ int64_t region_items(const Region &R, int64_t w) {
    int64_t total = 0;
    for (int64_t a0 = R.A0; a0 < R.A1; a0 += w) {
        int64_t c1, c2;
        tile_counts(R, a0, a0 + w < R.A1 ? a0 + w : R.A1, c1, c2);
        total += c1 + c2;
    }
    return total;
}

__device__ __forceinline__ void region_item(const Region &R, int64_t w, int64_t k, int64_t &a, int64_t &b) {
    for (int64_t a0 = R.A0; a0 < R.A1; a0 += w) {
        const int64_t a1 = a0 + w < R.A1 ? a0 + w : R.A1;
        int64_t c1, c2;
        tile_counts(R, a0, a1, c1, c2);
        if (k >= c1 + c2) { k -= c1 + c2; continue; }
        const int64_t bs = R.B0 > a0 + 1 ? R.B0 : a0 + 1;
        if (k < c1) {
            // largest m = b - a0 with tri2(m) <= k + tri2(bs - a0)
            const int64_t key = k + tri2(bs - a0);
            int64_t m = (int64_t)floor((1.0 + sqrt(1.0 + 8.0 * (double)key)) * 0.5);
            while (m > 0 && tri2(m) > key) --m;
            while (tri2(m + 1) <= key) ++m;
            b = a0 + m;
            a = a0 + (key - tri2(m));
        } else {
            const int64_t r = k - c1, ww = a1 - a0;
            const int64_t b2 = bs > a1 ? bs : a1;
            b = b2 + r / ww;
            a = a0 + r % ww;
        }
        return;
    }
    a = 0;
    b = 0;
}

// One support class of the pairwise matrix.  The class's items are split
// into kXcdQueues contiguous ranges with a work-queue counter each; a
// workgroup drains the range of its own XCD first (workgroups are dealt to
// the XCDs round-robin by index), then helps the others, so each XCD works
// on a few tiles at a time and their objects stay in its L2.
constexpr int kXcdQueues = 8;

template <int CLS, typename TIn, int START>
__global__ __launch_bounds__(ShapeCfg<CLS>::threads, ShapeCfg<CLS>::occ) void k_pairwise_q(
    KSet X, KOpts o, void *ws, int cls, int chunk, int tile, double *out, int32_t *status) {
    constexpr int G = ShapeCfg<CLS>::G, GS = ShapeCfg<CLS>::GS, NG = ShapeCfg<CLS>::groups;
    constexpr bool LT = ShapeCfg<CLS>::LT;
    __shared__ GroupMem<G, GS> mem[NG];
    __shared__ TileOf<CLS, START> tiles[NG];
    const int tid = threadIdx.x;
    const int g = tid / G, l = tid % G, gbase = (tid & 63) & ~(G - 1);
    SortWS s = sort_ws(ws);
    const int64_t n = X.n, n16 = s.bounds[0], n32 = s.bounds[1];
    const Region R = class_region(cls, n16, n32, n);
    const int64_t w = tile_width(R, tile);
    const int64_t items = region_items(R, w);
    GroupMem<G, GS> &M = mem[g];
    const int home = (int)(blockIdx.x % kXcdQueues);
#pragma unroll 1
    for (int q = 0; q < kXcdQueues; ++q) {
        const int x = (home + q) % kXcdQueues;
        const int64_t lo = items * x / kXcdQueues, hi = items * (x + 1) / kXcdQueues;
#pragma unroll 1
        for (;;) {
            if (l == 0)
                M.grab = (long long)atomicAdd(&s.counters[cls * kXcdQueues + x], (unsigned long long)chunk);
            wsync();
            const int64_t base = lo + M.grab;
            wsync();
            if (base >= hi) break;
            const int64_t end = base + chunk < hi ? base + chunk : hi;
            for (int64_t k = base; k < end; ++k) {
                int64_t a, b;
                region_item(R, w, k, a, b);
                const int64_t pi = s.perm[a], pj = s.perm[b];
                const int64_t lo2 = pi < pj ? pi : pj, hi2 = pi < pj ? pj : pi;
                NodeState<G, GS, LT> N;
                PairView pv = orient(X, lo2, X, hi2, (int)sizeof(TIn));
                SolveOut r = solve_pair<G, GS, LT, TIn, START>(M, tiles[g], N, pv, X.d, o, l, gbase);
                if (l == 0) {
                    const int64_t idx = condensed_index(n, lo2, hi2);
                    out[idx] = r.status == kOk ? r.d2 : __builtin_nan("");
                    if (status) status[idx] = r.status;
                }
            }
        }
    }
}

// Row i of the strict upper triangle holds n-1-i pairs; k -> (i, j).
__device__ __forceinline__ void condensed_ij(int64_t n, int64_t k, int64_t &i, int64_t &j) {
    const double nn = (double)n;
    const double disc = (2.0 * nn - 1.0) * (2.0 * nn - 1.0) - 8.0 * (double)k;
    int64_t r = (int64_t)floor(((2.0 * nn - 1.0) - sqrt(disc > 0.0 ? disc : 0.0)) * 0.5);
    if (r < 0) r = 0;
    if (r > n - 2) r = n - 2;
    while (r > 0 && r * n - r * (r + 1) / 2 > k) --r;
    while (r + 1 <= n - 2 && (r + 1) * n - (r + 1) * (r + 2) / 2 <= k) ++r;
    i = r;
    j = k - (r * n - r * (r + 1) / 2) + r + 1;
}

// Plain schedule: one shape for every pair, pairs in input order.
template <int CLS, typename TIn, int START>
__global__ __launch_bounds__(ShapeCfg<CLS>::threads, ShapeCfg<CLS>::occ) void k_pairwise_plain(KSet X, KOpts o, double *out,
                                                                           int32_t *status) {
    constexpr int G = ShapeCfg<CLS>::G, GS = ShapeCfg<CLS>::GS, NG = ShapeCfg<CLS>::groups;
    constexpr bool LT = ShapeCfg<CLS>::LT;
    __shared__ GroupMem<G, GS> mem[NG];
    __shared__ TileOf<CLS, START> tiles[NG];
    const int tid = threadIdx.x;
    const int g = tid / G, l = tid % G, gbase = (tid & 63) & ~(G - 1);
    const int64_t m = X.n * (X.n - 1) / 2;
    const int64_t stride = (int64_t)gridDim.x * NG;
    for (int64_t k = (int64_t)blockIdx.x * NG + g; k < m; k += stride) {
        int64_t i, j;
        condensed_ij(X.n, k, i, j);
        NodeState<G, GS, LT> N;
        PairView pv = orient(X, i, X, j, (int)sizeof(TIn));
        SolveOut r = solve_pair<G, GS, LT, TIn, START>(mem[g], tiles[g], N, pv, X.d, o, l, gbase);
        if (l == 0) {
            out[k] = r.status == kOk ? r.d2 : __builtin_nan("");
            if (status) status[k] = r.status;
        }
    }
}

// ------------------------------------------------------------ cost tiles

template <typename TIn>
__global__ void k_cost_tiles_f64(KSet A, KSet B, const int64_t *pairs, int64_t npairs,
                                 double *tiles, const int64_t *tile_off) {
    for (int64_t k = blockIdx.x; k < npairs; k += gridDim.x) {
        const int64_t i = pairs[2 * k], j = pairs[2 * k + 1];
        if (i < 0 || i >= A.n || j < 0 || j >= B.n) continue;
        const int64_t a0 = A.off[i], t = A.off[i + 1] - a0;
        const int64_t b0 = B.off[j], s = B.off[j + 1] - b0;
        if (t < 1 || s < 1 || t > D2_MAX_SUPPORT || s > D2_MAX_SUPPORT) continue;
        const TIn *x = (const TIn *)A.pts + a0 * A.d;
        const TIn *y = (const TIn *)B.pts + b0 * B.d;
        double *dst = tiles + tile_off[k];
        for (int64_t c = threadIdx.x; c < t * s; c += blockDim.x) {
            const int64_t a = c / s, b = c % s;
            double acc = 0.0;
            for (int q = 0; q < A.d; ++q) {
                const double diff = (double)x[a * A.d + q] - (double)y[b * B.d + q];
                acc = fma(diff, diff, acc);
            }
            dst[c] = acc;
        }
    }
}

// ------------------------------------------------------- BF16 cost tiles

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kBfSteps = 16;      // MFMA k-steps (8 coordinates each) held in registers

__device__ __forceinline__ unsigned short f32_to_bf16(float f) {  // round to nearest even
    unsigned int u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (unsigned short)((u >> 16) | 0x40u);  // NaN stays NaN
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
    return __uint_as_float((unsigned int)h << 16);
}

// MFMA operand fragments (v_mfma_f32_32x32x8_bf16) of one object's atoms for
// coordinates [kc, kc + 8 kBfSteps): lane l supplies atom (l mod 32) and, at
// step m, coordinates kc + 8m + 4(l div 32) .. +3, rounded FP32 -> BF16;
// `norm` accumulates the squares of the rounded values in FP32, in that
// order.  The same fragment serves as the A operand (atoms as rows) or the B
// operand (atoms as columns).  All loads are issued before any rounding.
template <typename TIn>
__device__ __forceinline__ void bf16_frags(const TIn *pts, int natoms, int d, int kc,
                                           bf16x4 (&f)[kBfSteps], float &norm) {
    const int l = threadIdx.x & 63, r = l & 31, h = l >> 5;
    const bool ok = r < natoms;
    const TIn *p = pts + (int64_t)(ok ? r : 0) * d;
    float v[kBfSteps][4];
    const bool vec = ((d & 3) == 0) && ((((uintptr_t)pts) & 15) == 0);
    if (vec) {
#pragma unroll
        for (int m = 0; m < kBfSteps; ++m) {
            const int k = kc + 8 * m + 4 * h;
            if constexpr (sizeof(TIn) == 4) {
                const float4 t = (ok && k < d) ? *(const float4 *)(p + k) : make_float4(0.f, 0.f, 0.f, 0.f);
                v[m][0] = t.x; v[m][1] = t.y; v[m][2] = t.z; v[m][3] = t.w;
            } else {
                const double2 z2 = make_double2(0.0, 0.0);
                const double2 t0 = (ok && k < d) ? *(const double2 *)(p + k) : z2;
                const double2 t1 = (ok && k < d) ? *(const double2 *)(p + k + 2) : z2;
                v[m][0] = (float)t0.x; v[m][1] = (float)t0.y; v[m][2] = (float)t1.x; v[m][3] = (float)t1.y;
            }
        }
    } else {
#pragma unroll
        for (int m = 0; m < kBfSteps; ++m)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = kc + 8 * m + 4 * h + q;
                v[m][q] = (ok && k < d) ? (float)p[k] : 0.f;
            }
    }
#pragma unroll
    for (int m = 0; m < kBfSteps; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const unsigned short b = f32_to_bf16(v[m][q]);
            const float fq = bf16_to_f32(b);
            norm = fmaf(fq, fq, norm);
            f[m][q] = (short)b;
        }
}

// acc += rows . cols over the steps of one coordinate round.
__device__ __forceinline__ void bf16_mma(const bf16x4 (&rows)[kBfSteps], const bf16x4 (&cols)[kBfSteps],
                                         int steps, f32x16 &acc) {
#pragma unroll
    for (int m = 0; m < kBfSteps; ++m)
        if (m < steps) acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(rows[m], cols[m], acc, 0, 0, 0);
}

// C_ab = max(0, |row a|^2 + |col b|^2 - 2 acc_ab) into a row-major 32 x 32
// tile.  Accumulator j of lane l is entry (8 (j div 4) + 4 (l div 32) +
// (j mod 4), l mod 32); rowN / colN are the squared norms of atom (l mod 32)
// on the row / column side.  NaN passes through the clamp, to be flagged.
__device__ __forceinline__ void bf16_epilogue(const f32x16 &acc, float rowN, float colN, float *out,
                                              float *lds32) {
    const int l = threadIdx.x & 63, r = l & 31, h = l >> 5;
    if (h == 0) lds32[r] = rowN;
    wsync();
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int row = (j >> 2) * 8 + h * 4 + (j & 3);
        const float c = (lds32[row] + colN) - 2.f * acc[j];
        out[row * 32 + r] = c < 0.f ? 0.f : c;
    }
    wsync();
}

// The centroids as BF16 MFMA fragments, once per call (d <= 8 kBfSteps):
// fragment m of lane l of centroid j at zf[(j kBfSteps + m) 64 + l] (the
// layout bf16_frags forms), and the squared norms of its atoms (from the
// same rounded values) at zn[32 j + atom].  One wavefront per centroid.
template <typename TIn>
__global__ __launch_bounds__(256) void k_bf16_centroid_frags(KSet Z, bf16x4 *zf, float *zn) {
    const int lane = threadIdx.x & 63;
    for (int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); j < Z.n; j += (int64_t)gridDim.x * 4) {
        const int64_t b0 = Z.off[j];
        const int s = (int)(Z.off[j + 1] - b0);
        bf16x4 f[kBfSteps];
        float nz = 0.f;
        bf16_frags<TIn>((const TIn *)Z.pts + b0 * Z.d, s >= 1 && s <= 32 ? s : 0, Z.d, 0, f, nz);
#pragma unroll
        for (int m = 0; m < kBfSteps; ++m) zf[(j * kBfSteps + m) * 64 + lane] = f[m];
        nz += __shfl_xor(nz, 32, 64);
        if (lane < 32) zn[j * 32 + lane] = nz;
    }
}

// One pair's cost tile, transposed: A = the column atoms, B = the row atoms,
// so accumulator j of lane l holds row (l mod 32), column 8 (j div 4) +
// 4 (l div 32) + (j mod 4).  With CACHED (d <= 8 kBfSteps) the object's
// fragments and atom norms come from LDS (xf, xn) and the centroid's from
// the per-call fragments (zf, zn); otherwise both sides are formed here.
// `rown` receives the squared norm of row atom (l mod 32); the column norms
// go to cn[0..32).  All 64 lanes take part.
template <typename TIn, bool CACHED>
__device__ __forceinline__ void bf16_tile_rows(const PairView &pv, int d, const bf16x4 (*xf)[64],
                                               const float *xn, const bf16x4 *zf, const float *zn,
                                               f32x16 &acc, float &rown, float *cn) {
    const int lane = threadIdx.x & 63;
    if constexpr (CACHED) {
        // X is the column side when the pair is swapped (rows = the centroid)
        const bool xcol = pv.swapped;
        const int steps = (d + 7) / 8;
#pragma unroll
        for (int m = 0; m < kBfSteps; ++m) {
            if (m < steps) {
                const bf16x4 fz = zf[m * 64 + lane], fx = xf[m][lane];
                acc = xcol ? __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(fx, fz, acc, 0, 0, 0)
                           : __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(fz, fx, acc, 0, 0, 0);
            }
        }
        const float nx = xn[lane & 31], nz = zn[lane & 31];
        if (lane < 32) cn[lane] = xcol ? nx : nz;
        rown = xcol ? nz : nx;
    } else {
        float ncol = 0.f, nrow = 0.f;
        for (int kc = 0; kc < d; kc += 8 * kBfSteps) {
            bf16x4 fc[kBfSteps], fr[kBfSteps];
            bf16_frags<TIn>((const TIn *)pv.xc, pv.S, d, kc, fc, ncol);
            bf16_frags<TIn>((const TIn *)pv.xr, pv.T, d, kc, fr, nrow);
            bf16_mma(fc, fr, (d - kc + 7) / 8, acc);
        }
        ncol += __shfl_xor(ncol, 32, 64);
        nrow += __shfl_xor(nrow, 32, 64);
        if (lane < 32) cn[lane] = ncol;
        rown = nrow;
    }
}

// BF16 cost mode: the labelling of k_assign in the 32-lane shape, each
// wavefront computing the cost tiles of its two pairs with MFMA right
// before solving them, so no tile leaves the chip.  The row's object is
// rounded to BF16 fragments once per item, into LDS, and the centroids'
// fragments were formed once per call (k_bf16_centroid_frags) when d <= 8
// kBfSteps.  Wave w takes
// centroids j0 + 2w (its first group) and j0 + 2w + 1 (its second), then
// steps by the workgroup's group count.  The tiles come out transposed
// (bf16_tile_rows): lane l holds half of row (l mod 32) of pair (l div 32)
// and half of the same row of the other pair, so one exchange with lane
// l ^ 32 gives every lane its whole cost row, written straight into the
// solver's register row: C = max(0, |row|^2 + |col|^2 - 2 acc).
template <typename TIn, int START, bool CACHED>
__global__ __launch_bounds__(ShapeCfg<1>::threads, ShapeCfg<1>::occ) void k_assign_bf16(
    KSet X, KSet Z, KOpts o, int64_t chunks, int64_t per_chunk, int32_t *labels, double *best, double *all,
    int32_t *row_status, double *ws_best, int32_t *ws_label, int32_t *ws_status, const bf16x4 *zfrag,
    const float *znorm) {
    constexpr int G = ShapeCfg<1>::G, GS = ShapeCfg<1>::GS, NG = ShapeCfg<1>::groups;
    constexpr bool LT = ShapeCfg<1>::LT;
    static_assert(G == 32 && GS == 32 && !LT, "two pairs of up to 32 atoms per wavefront");
    __shared__ GroupMem<G, GS> mem[NG];
    __shared__ TileOf<1, START> ltile[NG];
    __shared__ float cnorm[NG][32];
    __shared__ bf16x4 xfrag[kBfSteps][64];
    __shared__ float xnorm[32];
    __shared__ double red_v[NG];
    __shared__ int red_i[NG], red_s[NG];
    const int tid = threadIdx.x;
    const int g = tid / G, l = tid % G, gbase = (tid & 63) & ~(G - 1);
    const int w = tid >> 6, h = (tid >> 5) & 1;
    const int d = X.d;
    const int64_t total = X.n * chunks;
    const int64_t K = Z.n;
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int64_t i = item / chunks, ch = item % chunks;
        const int64_t j0 = ch * per_chunk;
        const int64_t j1 = j0 + per_chunk < K ? j0 + per_chunk : K;
        const int64_t a0 = X.off[i];
        const int tx = (int)(X.off[i + 1] - a0);
        const bool xc = CACHED && tx >= 1 && tx <= 32;
        if (xc && w == 0) {
            bf16x4 f[kBfSteps];
            float nx = 0.f;
            bf16_frags<TIn>((const TIn *)X.pts + a0 * d, tx, d, 0, f, nx);
#pragma unroll
            for (int m = 0; m < kBfSteps; ++m) xfrag[m][tid] = f[m];
            nx += __shfl_xor(nx, 32, 64);
            if (tid < 32) xnorm[tid] = nx;
        }
        __syncthreads();
        double bv = INFINITY;
        int bj = kNoKey, worst = kOk;
        for (int64_t jp = j0 + 2 * w; jp < j1; jp += NG) {   // wave-uniform
            const bool hasB = jp + 1 < j1;
            const PairView pa = orient(X, i, Z, jp, (int)sizeof(TIn));
            const PairView pb = hasB ? orient(X, i, Z, jp + 1, (int)sizeof(TIn)) : pa;
            const bool okA = pa.T >= 1 && pa.S >= 1 && pa.T <= 32 && pa.S <= 32;
            const bool okB = hasB && pb.T >= 1 && pb.S >= 1 && pb.T <= 32 && pb.S <= 32;
            f32x16 accA = {}, accB = {};
            float rnA = 0.f, rnB = 0.f;
            // (with CACHED, a pair is only solved when the object's fragments are in LDS)
            if (okA && (!CACHED || xc))
                bf16_tile_rows<TIn, CACHED>(pa, d, xfrag, xnorm, zfrag + jp * kBfSteps * 64, znorm + jp * 32,
                                            accA, rnA, cnorm[2 * w]);
            if (okB && (!CACHED || xc))
                bf16_tile_rows<TIn, CACHED>(pb, d, xfrag, xnorm, zfrag + (jp + 1) * kBfSteps * 64,
                                            znorm + (jp + 1) * 32, accB, rnB, cnorm[2 * w + 1]);
            wsync();
            // lane l keeps its own pair's half row; the other half comes from
            // lane l ^ 32, which holds it for the pair it does not solve
            NodeState<G, GS, LT> N;
            const PairView pv = h ? pb : pa;
            const bool hasR = l < pv.T;
            const float rn = h ? rnB : rnA;
            const float *cn = cnorm[g];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const float own = h ? accB[q] : accA[q];
                const float got = __shfl_xor(h ? accA[q] : accB[q], 32, 64);
                const float lo = h ? got : own;   // column 8 (q div 4) + (q mod 4)
                const float hi = h ? own : got;   // column 8 (q div 4) + 4 + (q mod 4)
                const int c0 = 8 * (q >> 2) + (q & 3), c1 = c0 + 4;
                const float v0 = (rn + cn[c0]) - 2.f * lo, v1 = (rn + cn[c1]) - 2.f * hi;
                // NaN passes through the clamp, to be flagged by the solver
                N.crow[c0] = (hasR && c0 < pv.S) ? (double)(v0 < 0.f ? 0.f : v0) : INFINITY;
                N.crow[c1] = (hasR && c1 < pv.S) ? (double)(v1 < 0.f ? 0.f : v1) : INFINITY;
            }
            wsync();   // the column norms are read before the next round writes them
            const int64_t j = jp + h;
            if (h == 0 || hasB) {
                SolveOut res = solve_pair<G, GS, LT, TIn, START>(mem[g], ltile[g], N, pv, d, o, l, gbase, nullptr,
                                                                 0, 0, true);
                if (res.status != kOk) {
                    worst = res.status > worst ? res.status : worst;
                    res.d2 = __builtin_nan("");
                } else if (res.d2 < bv || (res.d2 == bv && (int)j < bj)) {
                    bv = res.d2;
                    bj = (int)j;
                }
                if (all && l == 0) all[i * K + j] = res.d2;
            }
        }
        if (l == 0) { red_v[g] = bv; red_i[g] = bj; red_s[g] = worst; }
        __syncthreads();
        if (tid == 0) {
            double v = INFINITY;
            int jj = kNoKey, st = kOk;
            for (int q = 0; q < NG; ++q) {
                if (red_v[q] < v || (red_v[q] == v && red_i[q] < jj)) { v = red_v[q]; jj = red_i[q]; }
                st = red_s[q] > st ? red_s[q] : st;
            }
            if (chunks == 1) {
                labels[i] = st == kOk ? jj : -1;
                best[i] = st == kOk ? v : __builtin_nan("");
                if (row_status) row_status[i] = st;
            } else {
                ws_best[i * chunks + ch] = v;
                ws_label[i * chunks + ch] = jj;
                ws_status[i * chunks + ch] = st;
            }
        }
        __syncthreads();
    }
}

// Explicit pairs into caller tiles (FP64, caller orientation t_i x s_j).
template <typename TIn>
__global__ __launch_bounds__(256) void k_cost_bf16_pairs(KSet A, KSet B, const int64_t *pairs,
                                                         int64_t npairs, double *tiles,
                                                         const int64_t *tile_off) {
    __shared__ float lds[4][32];
    __shared__ float tl[4][1024];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int d = A.d;
    for (int64_t k = (int64_t)blockIdx.x * 4 + w; k < npairs; k += (int64_t)gridDim.x * 4) {
        const int64_t i = pairs[2 * k], j = pairs[2 * k + 1];
        if (i < 0 || i >= A.n || j < 0 || j >= B.n) continue;
        const int64_t a0 = A.off[i], b0 = B.off[j];
        const int t = (int)(A.off[i + 1] - a0), s = (int)(B.off[j + 1] - b0);
        if (t < 1 || s < 1 || t > 32 || s > 32) continue;
        const TIn *pa = (const TIn *)A.pts + a0 * d;
        const TIn *pb = (const TIn *)B.pts + b0 * d;
        const bool sw = t < s;
        f32x16 acc = {};
        float na = 0.f, nb = 0.f;
        for (int kc = 0; kc < d; kc += 8 * kBfSteps) {
            bf16x4 fa[kBfSteps], fb[kBfSteps];
            bf16_frags<TIn>(pa, t, d, kc, fa, na);
            bf16_frags<TIn>(pb, s, d, kc, fb, nb);
            const int steps = (d - kc + 7) / 8;
            if (sw) bf16_mma(fb, fa, steps, acc);
            else bf16_mma(fa, fb, steps, acc);
        }
        na += __shfl_xor(na, 32, 64);
        nb += __shfl_xor(nb, 32, 64);
        bf16_epilogue(acc, sw ? nb : na, sw ? na : nb, tl[w], lds[w]);
        double *dst = tiles + tile_off[k];
        const int T = sw ? s : t, S = sw ? t : s;   // oriented sizes
        for (int c = l; c < T * S; c += 64) {
            const int a = c / S, b = c % S;      // oriented row a, column b
            const double v = (double)tl[w][a * 32 + b];
            if (!sw) dst[(int64_t)a * S + b] = v;
            else dst[(int64_t)b * T + a] = v;
        }
        wsync();
    }
}

// ------------------------------------------------------------ launchers


int class_for(int maxsup_a, int maxsup_b) {
    const int T = maxsup_a > maxsup_b ? maxsup_a : maxsup_b;
    const int S = maxsup_a < maxsup_b ? maxsup_a : maxsup_b;
    return class_of(T, S);
}

int class_groups(int cls) {
    switch (cls) {
    case 0: return ShapeCfg<0>::groups;
    case 1: return ShapeCfg<1>::groups;
    case 2: return ShapeCfg<2>::groups;
    default: return ShapeCfg<3>::groups;
    }
}

int class_threads(int cls) {
    switch (cls) {
    case 0: return ShapeCfg<0>::threads;
    case 1: return ShapeCfg<1>::threads;
    case 2: return ShapeCfg<2>::threads;
    default: return ShapeCfg<3>::threads;
    }
}

// ---- labelling

constexpr int kXcds = 8;                        // XCDs of the MI355X, each with its own L2
constexpr size_t kXcdSplitBytes = 1u << 20;     // a quarter of one XCD's 4 MiB L2

AssignPlan plan_assign(const KSet &X, const KSet &Z, int xmax, int zmax, int cu_count, int schedule,
                       int cost_mode) {
    AssignPlan p;
    p.bf16 = cost_mode == D2_COST_BF16_MFMA;
    p.plain = schedule == D2_SCHED_PLAIN && !p.bf16;
    // classes the rows can fall in: rows of support 1..xmax against zmax
    const int cmin = class_for(1, zmax), cmax = class_for(xmax, zmax);
    p.binned = !p.plain && !p.bf16 && cmin != cmax;
    // BF16 mode: the fused kernel in the 32-lane shape (supports <= 32)
    p.single_class = p.plain ? 3 : (p.bf16 ? 1 : cmax);
    const int NG = class_groups(p.single_class);
    const int64_t K = Z.n > 0 ? Z.n : 1;
    const int64_t target = (int64_t)(cu_count > 0 ? cu_count : 256) * 8;
    int64_t chunks = X.n > 0 ? (target + X.n - 1) / X.n : 1;
    // XCD-aware split.  Workgroups are dealt to the 8 XCDs round-robin by
    // index, and item = row * chunks + chunk, so with a multiple of 8 chunks
    // every workgroup of one XCD works on the same eighth of the centroids,
    // which then stays in that XCD's L2 instead of streaming from HBM once
    // per row.  Used when the centroid points (bounded by K x max support x
    // d) are more than a quarter of one L2.
    const size_t zbytes = (size_t)K * (size_t)(zmax > 0 ? zmax : 1) * (size_t)(Z.d > 0 ? Z.d : 1) *
                          (Z.dtype == D2_F32 ? 4u : 8u);
    if (zbytes > kXcdSplitBytes) chunks = ((chunks + kXcds - 1) / kXcds) * kXcds;
    const int64_t max_chunks = (K + NG - 1) / NG;
    if (chunks > max_chunks) chunks = max_chunks;
    if (chunks < 1) chunks = 1;
    p.chunks = chunks;
    p.per_chunk = (K + chunks - 1) / chunks;
    p.part_bytes = chunks > 1 ? (size_t)X.n * chunks * (sizeof(double) + 2 * sizeof(int32_t)) : 0;
    p.sort_bytes = p.binned ? sort_ws_bytes(X.n) : 0;
    // BF16 mode: the centroids as MFMA fragments (8 KiB each) and atom norms
    p.frag_bytes = (p.bf16 && Z.d <= 8 * kBfSteps) ? (size_t)K * (kBfSteps * 64 * 8 + 32 * 4) : 0;
    p.ws_bytes = p.part_bytes + p.sort_bytes + p.frag_bytes;
    p.zmax = zmax;
    return p;
}

struct AssignRun {
    const LaunchCtx &c;
    const AssignPlan &p;
    const KSet &X, &Z;
    const KOpts &o;
    int32_t *labels; double *best; double *all; int32_t *row_status;
    double *wb; int32_t *wl, *wsn;
    const int64_t *perm, *bounds;
    int cls_idx;
    int64_t grid;
    int64_t row_begin, row_end;
    const bf16x4 *zfrag;
    const float *znorm;
    template <int C, typename TIn, int V>
    hipError_t run() {
        if (p.bf16) {
            if constexpr (C == 1) {
                if (zfrag)
                    hipLaunchKernelGGL((k_assign_bf16<TIn, V, true>), dim3((unsigned)grid),
                                       dim3(ShapeCfg<1>::threads), 0, c.stream, X, Z, o, p.chunks, p.per_chunk,
                                       labels, best, all, row_status, wb, wl, wsn, zfrag, znorm);
                else
                    hipLaunchKernelGGL((k_assign_bf16<TIn, V, false>), dim3((unsigned)grid),
                                       dim3(ShapeCfg<1>::threads), 0, c.stream, X, Z, o, p.chunks, p.per_chunk,
                                       labels, best, all, row_status, wb, wl, wsn, zfrag, znorm);
            } else {
                return hipErrorInvalidValue;
            }
        } else {
            hipLaunchKernelGGL((k_assign<C, TIn, V>), dim3((unsigned)grid), dim3(ShapeCfg<C>::threads), 0,
                               c.stream, X, Z, o, perm, bounds, cls_idx, row_begin, row_end, p.chunks,
                               p.per_chunk, labels, best, all, row_status, wb, wl, wsn);
        }
        return hipGetLastError();
    }
};

hipError_t launch_assign(const LaunchCtx &c, const AssignPlan &p, const KSet &X, const KSet &Z,
                         const KOpts &o, int32_t *labels, double *best, double *all,
                         int32_t *row_status, void *ws) {
    if (X.n == 0) return hipSuccess;
    const bool f32 = X.dtype == D2_F32;
    const int start = o.init;
    double *wb = nullptr;
    int32_t *wl = nullptr, *wsn = nullptr;
    if (p.chunks > 1) {
        wb = (double *)ws;
        wl = (int32_t *)(wb + X.n * p.chunks);
        wsn = wl + X.n * p.chunks;
    }
    hipError_t e = hipSuccess;
    const int64_t items = X.n * p.chunks;
    if (!p.binned) {
        const bf16x4 *zfrag = nullptr;
        const float *znorm = nullptr;
        if (p.frag_bytes > 0) {
            bf16x4 *zf = (bf16x4 *)((char *)ws + p.part_bytes + p.sort_bytes);
            float *zn = (float *)(zf + Z.n * kBfSteps * 64);
            const int64_t fg = (Z.n + 3) / 4 < 65536 ? (Z.n + 3) / 4 : 65536;
            if (f32)
                hipLaunchKernelGGL(k_bf16_centroid_frags<float>, dim3((unsigned)fg), dim3(256), 0, c.stream, Z,
                                   zf, zn);
            else
                hipLaunchKernelGGL(k_bf16_centroid_frags<double>, dim3((unsigned)fg), dim3(256), 0, c.stream, Z,
                                   zf, zn);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            zfrag = zf;
            znorm = zn;
        }
        const int64_t grid = items < (1LL << 30) ? items : (1LL << 30);
        AssignRun r{c, p, X, Z, o, labels, best, all, row_status, wb, wl, wsn, nullptr, nullptr, 0, grid,
                    0, X.n, zfrag, znorm};
        e = dispatch_class(p.single_class, f32, start, r);
    } else {
        void *sws = (char *)ws + p.part_bytes;
        SortWS hs;  // host view of the device pointers
        {
            int64_t *q = (int64_t *)sws;
            hs.hist = q; hs.cursor = q + 66; hs.bounds = q + 132;
            hs.counters = (unsigned long long *)(q + 140); hs.perm = q + 172;
        }
        const int sb = (int)((X.n + 255) / 256 < 1024 ? (X.n + 255) / 256 : 1024);
        hipLaunchKernelGGL(k_sort_init, dim3(1), dim3(128), 0, c.stream, sws);
        hipLaunchKernelGGL(k_sort_hist, dim3(sb), dim3(256), 0, c.stream, X, sws);
        hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(64), 0, c.stream, sws, X.n, 1, p.zmax, 16, 32);
        hipLaunchKernelGGL(k_sort_scatter, dim3(sb), dim3(256), 0, c.stream, X, sws);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // every class a row can fall in; kernels of empty classes exit at once
        for (int cls = class_for(1, p.zmax); cls < 4 && e == hipSuccess; ++cls) {
            const int64_t grid = (int64_t)(c.cu_count > 0 ? c.cu_count : 256) * 16;
            const int64_t g2 = items < grid ? (items > 0 ? items : 1) : grid;
            AssignRun r{c, p, X, Z, o, labels, best, all, row_status, wb, wl, wsn, hs.perm, hs.bounds,
                        cls, g2, 0, X.n, nullptr, nullptr};
            e = dispatch_class(cls, f32, start, r);
        }
    }
    if (e != hipSuccess || p.chunks == 1) return e;
    const int64_t blocks = (X.n + 255) / 256;
    hipLaunchKernelGGL(k_assign_reduce, dim3((unsigned)blocks), dim3(256), 0, c.stream, X.n, p.chunks,
                       wb, wl, wsn, labels, best, row_status);
    return hipGetLastError();
}

// ---- explicit pairs

struct EmdRun {
    const LaunchCtx &c;
    const KSet &A, &B;
    const int64_t *pairs; int64_t npairs;
    const KOpts &o;
    double *dist; const int64_t *plan_off; double *plan; const int64_t *dual_off; double *duals;
    int32_t *status, *pivots;
    template <int C, typename TIn, int V>
    hipError_t run() {
        const int NG = ShapeCfg<C>::groups;
        int64_t grid = (npairs + NG - 1) / NG;
        if (grid > (1LL << 30)) grid = 1LL << 30;
        hipLaunchKernelGGL((k_emd_pairs<C, TIn, V>), dim3((unsigned)grid), dim3(ShapeCfg<C>::threads), 0,
                           c.stream, A, B, pairs, npairs, o, dist, plan_off, plan, dual_off, duals, status,
                           pivots);
        return hipGetLastError();
    }
};

hipError_t launch_emd_pairs(const LaunchCtx &c, int cls, const KSet &A, const KSet &B,
                            const int64_t *pairs, int64_t npairs, const KOpts &o, double *dist,
                            const int64_t *plan_off, double *plan, const int64_t *dual_off,
                            double *duals, int32_t *status, int32_t *pivots) {
    if (npairs == 0) return hipSuccess;
    EmdRun r{c, A, B, pairs, npairs, o, dist, plan_off, plan, dual_off, duals, status, pivots};
    return dispatch_class(cls, A.dtype == D2_F32, o.init, r);
}

// ---- pairwise

PairwisePlan plan_pairwise(const KSet &X, int xmax, int schedule) {
    PairwisePlan p;
    p.plain = schedule == D2_SCHED_PLAIN;
    p.plain_class = p.plain ? 3 : class_for(xmax, xmax);
    p.binned = !p.plain && class_for(xmax, xmax) != 0;
    p.ws_bytes = p.plain ? 0 : sort_ws_bytes(X.n);
    return p;
}

struct PairwisePlainRun {
    const LaunchCtx &c;
    const KSet &X; const KOpts &o; double *out; int32_t *status;
    template <int C, typename TIn, int V>
    hipError_t run() {
        const int NG = ShapeCfg<C>::groups;
        const int64_t m = X.n * (X.n - 1) / 2;
        int64_t grid = (m + NG - 1) / NG;
        if (grid > (1LL << 30)) grid = 1LL << 30;
        hipLaunchKernelGGL((k_pairwise_plain<C, TIn, V>), dim3((unsigned)grid), dim3(ShapeCfg<C>::threads),
                           0, c.stream, X, o, out, status);
        return hipGetLastError();
    }
};

struct PairwiseQRun {
    const LaunchCtx &c;
    const KSet &X; const KOpts &o; void *ws; int cls; int chunk; int tile; int64_t grid;
    double *out; int32_t *status;
    template <int C, typename TIn, int V>
    hipError_t run() {
        hipLaunchKernelGGL((k_pairwise_q<C, TIn, V>), dim3((unsigned)grid), dim3(ShapeCfg<C>::threads), 0,
                           c.stream, X, o, ws, cls, chunk, tile, out, status);
        return hipGetLastError();
    }
};

hipError_t launch_pairwise(const LaunchCtx &c, const PairwisePlan &p, const KSet &X, const KOpts &o,
                           double *condensed, int32_t *status, void *ws, const Schedule &sch, int only_class) {
    if (X.n < 2) return hipSuccess;
    const bool f32 = X.dtype == D2_F32;
    const int start = o.init;
    if (p.plain) {
        PairwisePlainRun r{c, X, o, condensed, status};
        return dispatch_class(p.plain_class, f32, start, r);
    }
    const int sb = (int)((X.n + 255) / 256 < 1024 ? (X.n + 255) / 256 : 1024);
    hipLaunchKernelGGL(k_sort_init, dim3(1), dim3(128), 0, c.stream, ws);
    hipLaunchKernelGGL(k_sort_hist, dim3(sb), dim3(256), 0, c.stream, X, ws);
    const int e0 = sch.edge[0] >= 1 && sch.edge[0] <= 16 ? sch.edge[0] : 16;
    const int e1 = sch.edge[1] >= e0 && sch.edge[1] <= 32 ? sch.edge[1] : 32;
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(64), 0, c.stream, ws, X.n, 0, 0, e0, e1);
    hipLaunchKernelGGL(k_sort_scatter, dim3(sb), dim3(256), 0, c.stream, X, ws);
    hipError_t e = hipGetLastError();
    // classes 0..3 (or the one asked for); empty ones exit at once
    for (int cls = 0; cls < 4 && e == hipSuccess; ++cls) {
        if (only_class >= 0 && cls != only_class) continue;
        const int per_cu = sch.blocks_per_cu[cls] > 0 ? sch.blocks_per_cu[cls] : 4;
        const int64_t grid = (int64_t)(c.cu_count > 0 ? c.cu_count : 256) * per_cu;
        PairwiseQRun r{c, X, o, ws, cls, sch.chunk[cls] > 0 ? sch.chunk[cls] : 4, sch.tile[cls], grid,
                       condensed, status};
        e = dispatch_class(cls, f32, start, r);
    }
    return e;
}

// ---- cost tiles

hipError_t launch_cost_tiles(const LaunchCtx &c, const KSet &A, const KSet &B,
                             const int64_t *pairs, int64_t npairs, int cost_mode, double *tiles,
                             const int64_t *tile_off) {
    if (npairs == 0) return hipSuccess;
    if (cost_mode == D2_COST_BF16_MFMA) {
        const int64_t g = (npairs + 3) / 4 < 65536 ? (npairs + 3) / 4 : 65536;
        if (A.dtype == D2_F32)
            hipLaunchKernelGGL(k_cost_bf16_pairs<float>, dim3((unsigned)g), dim3(256), 0, c.stream, A, B,
                               pairs, npairs, tiles, tile_off);
        else
            hipLaunchKernelGGL(k_cost_bf16_pairs<double>, dim3((unsigned)g), dim3(256), 0, c.stream, A, B,
                               pairs, npairs, tiles, tile_off);
        return hipGetLastError();
    }
    const int64_t grid = npairs < (1LL << 30) ? npairs : (1LL << 30);
    if (A.dtype == D2_F32)
        hipLaunchKernelGGL(k_cost_tiles_f64<float>, dim3((unsigned)grid), dim3(256), 0, c.stream, A, B,
                           pairs, npairs, tiles, tile_off);
    else
        hipLaunchKernelGGL(k_cost_tiles_f64<double>, dim3((unsigned)grid), dim3(256), 0, c.stream, A, B,
                           pairs, npairs, tiles, tile_off);
    return hipGetLastError();
}

}  // namespace d2
