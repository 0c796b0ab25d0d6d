// Centroid update of constrained D2-clustering (Alg. 2 Step 3*): Alg. 1 with
// the centroid weights held fixed, so that its LP separates into one
// transport problem per member (Sec. 2.2), for all clusters in one pass.
//
//   group    stable counting sort of the objects by label, in 64-object
//            tiles: per-(label, tile) counts, one exclusive scan over them
//            (label-major), then every tile places its objects with ballots.
//            Members of a cluster end up contiguous, in increasing index.
//   solve    Step 1: one lane group per member solves the transport problem
//            against the member's own centroid (the same solver as every
//            other entry point) and stores the basis tree as a cell list:
//            (member atom, centroid atom, flow) per tree edge.
//   mean     Step 2, Eq. (2): a cluster's members are cut into items of 64
//            (so one large cluster spreads over many workgroups).  In an
//            item's workgroup, member slices accumulate flow * coordinate
//            into private LDS rows, summed in slice order into the item's
//            partial numerators and flow totals; one workgroup per cluster
//            then adds its items in order, and each atom becomes numerator
//            over total flow.  No atomics anywhere, so repeated calls give
//            the same bits.
//   eps      Step 3: one wave per member evaluates its plan against the
//            moved atoms; the members' Step 1 and Step 3 values are summed
//            per item, then per cluster.
// Optional object weights (weighted D2-clustering, Eq. (3)-(4)) scale each
// member's flows in both sums of Eq. (4) and its terms of the objectives.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "d2_internal.h"
#include "d2_shapes.h"
#include "d2_solver.h"

namespace d2 {

namespace {

constexpr int kTile = 64;          // objects per tile of the counting sort
constexpr int kItem = 64;          // members per item of the mean and the sums
constexpr int kScanPer = 4096;     // entries per workgroup of the scan
constexpr int kUnlabelled = 5;     // D2_PAIR_UNLABELLED

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct UpdWS {
    int64_t *cnt;     // [(K+1) * tiles]: counts, then their exclusive prefix
    int64_t *bsum;    // [scan blocks]
    int64_t *perm;    // [n]: object of each sorted position
    int32_t *skey;    // [n]: its label (K for objects left out)
    double *d2m;      // [n]: Step 1 value of each sorted position
    double *eps3m;    // [n]: Step 3 value
    int32_t *stm;     // [n]: status
    int32_t *code;    // [n * cs]: (member atom << 16) | centroid atom, -1 = none
    double *flow;     // [n * cs]
    int64_t *itemoff; // [K+1]: first item of each cluster
    double *part;     // [items][zmax][d+1]: partial numerators, flow total last
    double *ie1, *ie3;   // [items]: partial objectives
    int64_t *icnt;    // [items]: members that entered Step 2
    const double *objw;  // caller's object weights (Eq. (3)), or null for 1
};

struct UpdDims {
    int64_t n, K, tiles, entries, sblocks, items;
    int cs, zmax, d;
};

UpdDims upd_dims(int64_t n, int64_t K, int d, int xmax, int zmax) {
    UpdDims u;
    u.n = n;
    u.K = K;
    u.tiles = n > 0 ? (n + kTile - 1) / kTile : 1;
    u.entries = (K + 1) * u.tiles;
    u.sblocks = (u.entries + kScanPer - 1) / kScanPer;
    // each cluster has ceil(n_j / kItem) <= n_j / kItem + 1 items
    u.items = (n > 0 ? (n + kItem - 1) / kItem : 0) + K;
    if (u.items < 1) u.items = 1;
    u.cs = xmax + zmax;
    u.zmax = zmax;
    u.d = d;
    return u;
}

size_t upd_layout(const UpdDims &u, void *base, UpdWS *w) {
    char *p = (char *)base;
    size_t off = 0;
    auto take = [&](size_t bytes) { char *q = p ? p + off : nullptr; off += align256(bytes); return q; };
    const int64_t n = u.n > 0 ? u.n : 1;
    UpdWS s;
    s.cnt = (int64_t *)take((size_t)u.entries * 8);
    s.bsum = (int64_t *)take((size_t)u.sblocks * 8);
    s.perm = (int64_t *)take((size_t)n * 8);
    s.skey = (int32_t *)take((size_t)n * 4);
    s.d2m = (double *)take((size_t)n * 8);
    s.eps3m = (double *)take((size_t)n * 8);
    s.stm = (int32_t *)take((size_t)n * 4);
    s.code = (int32_t *)take((size_t)n * u.cs * 4);
    s.flow = (double *)take((size_t)n * u.cs * 8);
    s.itemoff = (int64_t *)take((size_t)(u.K + 1) * 8);
    s.part = (double *)take((size_t)u.items * u.zmax * (u.d + 1) * 8);
    s.ie1 = (double *)take((size_t)u.items * 8);
    s.ie3 = (double *)take((size_t)u.items * 8);
    s.icnt = (int64_t *)take((size_t)u.items * 8);
    s.objw = nullptr;
    if (w) *w = s;
    return off;
}

__device__ __forceinline__ int64_t label_key(const int32_t *labels, int64_t i, int64_t K) {
    const int64_t j = labels[i];
    return (j >= 0 && j < K) ? j : K;
}

// Lanes of the wave below this one.
__device__ __forceinline__ uint64_t lanes_below() {
    const int l = threadIdx.x & 63;
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// ------------------------------------------------------------ grouping

__global__ void k_upd_fill(int64_t *p, int64_t m) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// One wave per tile: count[key][tile] = objects of the tile with that key.
__global__ void k_upd_count(const int32_t *labels, int64_t n, int64_t K, int64_t tiles, int64_t *cnt,
                            int32_t *obj_status) {
    const int64_t tile = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    if (tile >= tiles) return;
    const int64_t i = tile * kTile + (threadIdx.x & 63);
    const bool live = i < n;
    const int64_t key = live ? label_key(labels, i, K) : -1;
    if (live && key == K && obj_status) obj_status[i] = kUnlabelled;
    uint64_t todo = __ballot(live);
    while (todo) {   // one round per distinct key in the tile
        const int first = __builtin_ctzll(todo);
        const int64_t k0 = __shfl(key, first, 64);
        const uint64_t same = __ballot(live && key == k0);
        if ((threadIdx.x & 63) == first) cnt[k0 * tiles + tile] = __builtin_popcountll(same);
        todo &= ~same;
    }
}

// Exclusive prefix over cnt (label-major, tile-minor), in three steps.
__global__ void k_upd_scan_blocks(const int64_t *cnt, int64_t m, int64_t *bsum) {
    __shared__ int64_t part[256];
    const int64_t b0 = (int64_t)blockIdx.x * kScanPer;
    int64_t s = 0;
    for (int q = 0; q < kScanPer / 256; ++q) {
        const int64_t e = b0 + (int64_t)threadIdx.x * (kScanPer / 256) + q;
        if (e < m) s += cnt[e];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int q = 0; q < 256; ++q) t += part[q];
        bsum[blockIdx.x] = t;
    }
}

// Exclusive prefix of v[0, L) in place, by one workgroup of 1024 threads:
// contiguous chunks per thread, then a scan of the chunk sums in LDS.
__device__ void block_exclusive_scan(int64_t *v, int64_t L) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (L + 1023) / 1024;
    const int64_t b = t * chunk, e = b + chunk < L ? b + chunk : L;
    int64_t s = 0;
    for (int64_t q = b; q < e; ++q) s += v[q];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {   // inclusive Hillis-Steele scan
        const int64_t add = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    int64_t acc = t > 0 ? part[t - 1] : 0;
    for (int64_t q = b; q < e; ++q) {
        const int64_t x = v[q];
        v[q] = acc;
        acc += x;
    }
}

__global__ __launch_bounds__(1024) void k_upd_scan_top(int64_t *bsum, int64_t nb) {
    block_exclusive_scan(bsum, nb);
}

// Items per cluster (ceil of its members over kItem), then their prefix.
__global__ __launch_bounds__(1024) void k_upd_items(const int64_t *pre, int64_t K, int64_t tiles,
                                                    int64_t *itemoff) {
    for (int64_t j = threadIdx.x; j <= K; j += blockDim.x) {
        const int64_t cnt = j < K ? pre[(j + 1) * tiles] - pre[j * tiles] : 0;
        itemoff[j] = (cnt + kItem - 1) / kItem;
    }
    __syncthreads();
    block_exclusive_scan(itemoff, K + 1);
}

// Cluster of an item: the last j with itemoff[j] <= item (clusters without
// members own no items).
__device__ __forceinline__ int64_t item_cluster(const int64_t *itemoff, int64_t K, int64_t item) {
    int64_t lo = 0, hi = K;   // itemoff[lo] <= item < itemoff[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (itemoff[mid] <= item) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void k_upd_scan_apply(int64_t *cnt, int64_t m, const int64_t *bsum) {
    __shared__ int64_t part[256];
    constexpr int per = kScanPer / 256;
    const int64_t b0 = (int64_t)blockIdx.x * kScanPer;
    const int64_t e0 = b0 + (int64_t)threadIdx.x * per;
    int64_t v[per];
    int64_t s = 0;
    for (int q = 0; q < per; ++q) {
        v[q] = e0 + q < m ? cnt[e0 + q] : 0;
        s += v[q];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = bsum[blockIdx.x];
        for (int q = 0; q < 256; ++q) {
            const int64_t t = part[q];
            part[q] = acc;
            acc += t;
        }
    }
    __syncthreads();
    int64_t acc = part[threadIdx.x];
    for (int q = 0; q < per; ++q) {
        if (e0 + q < m) cnt[e0 + q] = acc;
        acc += v[q];
    }
}

// One wave per tile: each object goes to prefix[key][tile] + its rank among
// the tile's objects with the same key (stable).
__global__ void k_upd_place(const int32_t *labels, int64_t n, int64_t K, int64_t tiles, const int64_t *pre,
                            int64_t *perm, int32_t *skey) {
    const int64_t tile = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    if (tile >= tiles) return;
    const int64_t i = tile * kTile + (threadIdx.x & 63);
    const bool live = i < n;
    const int64_t key = live ? label_key(labels, i, K) : -1;
    int64_t pos = live ? pre[key * tiles + tile] : -1;   // all lanes' loads at once
    uint64_t todo = __ballot(live);
    while (todo) {
        const int first = __builtin_ctzll(todo);
        const int64_t k0 = __shfl(key, first, 64);
        const uint64_t same = __ballot(live && key == k0);
        if (live && key == k0) pos += __builtin_popcountll(same & lanes_below());
        todo &= ~same;
    }
    if (live) {
        perm[pos] = i;
        skey[pos] = (int32_t)key;
    }
}

// ------------------------------------------------------------ Step 1

// Sorted positions [0, members) are the labelled objects; the member count
// is the prefix of key K at tile 0.
template <int CLS, typename TIn, int START>
__global__ __launch_bounds__(ShapeCfg<CLS>::threads, ShapeCfg<CLS>::occ) void k_upd_solve(
    KSet X, KSet Z, KOpts o, int xmax, int zmax, UpdWS w, int64_t tiles, int cs, int32_t *obj_status) {
    constexpr int G = ShapeCfg<CLS>::G, GS = ShapeCfg<CLS>::GS, NG = ShapeCfg<CLS>::groups;
    constexpr bool LT = ShapeCfg<CLS>::LT;
    __shared__ GroupMem<G, GS> mem[NG];
    __shared__ TileOf<CLS, START> tiles_lds[NG];
    const int tid = threadIdx.x;
    const int g = tid / G, l = tid % G, gbase = (tid & 63) & ~(G - 1);
    const int64_t members = w.cnt[Z.n * tiles];
    const int64_t stride = (int64_t)gridDim.x * NG;
    for (int64_t m = (int64_t)blockIdx.x * NG + g; m < members; m += stride) {
        const int64_t i = w.perm[m], j = w.skey[m];
        const int64_t t = X.off[i + 1] - X.off[i], s = Z.off[j + 1] - Z.off[j];
        SolveOut r{kTooLarge, __builtin_nan("")};
        NodeState<G, GS, LT> N;
        PairView pv = orient(X, i, Z, j, (int)sizeof(TIn));
        // the cell list and the mean's LDS rows are sized by the declared bounds
        const double om = w.objw ? w.objw[i] : 1.0;
        if (!(om >= 0.0 && isfinite(om)))
            r.status = kBadWeights;
        else if (t >= 1 && s >= 1 && t <= xmax && s <= zmax)
            r = solve_pair<G, GS, LT, TIn, START>(mem[g], tiles_lds[g], N, pv, X.d, o, l, gbase);
        if (r.status == kOk) {
            const int T = pv.T, S = pv.S;
            int32_t *code = w.code + m * cs;
            double *flow = w.flow + m * cs;
            // edge of row node l to its parent column, then of column node l
            // to its parent row; the root has none
            if (l < T) {
                const int a = l, b = N.parR;
                code[l] = b < 0 ? -1 : (pv.swapped ? ((b << 16) | a) : ((a << 16) | b));
                flow[l] = b < 0 ? 0.0 : N.flowR;
            }
            if (l < S) {
                const int a = N.parC, b = l;
                code[T + l] = a < 0 ? -1 : (pv.swapped ? ((b << 16) | a) : ((a << 16) | b));
                flow[T + l] = a < 0 ? 0.0 : N.flowC;
            }
        }
        if (l == 0) {
            w.d2m[m] = r.status == kOk ? r.d2 : __builtin_nan("");
            w.stm[m] = r.status;
            if (obj_status) obj_status[i] = r.status;
        }
    }
}

// ------------------------------------------------------------ Step 2

// One workgroup of 256 per item (up to kItem members of one cluster).
// Thread (p, c), c < kb, p < P, adds flow * x[a][k0 + c] of the item's
// members m = lo + p, lo + p + P, ... into its own LDS accumulators
// acc[p][r][c], and the flows into acc[p][r][kb]; the slices are then summed
// in order into the item's partial row.
template <typename TIn>
__global__ __launch_bounds__(256) void k_upd_partial(KSet X, KSet Z, UpdWS w, int64_t tiles, int cs, int kb,
                                                      int P, int zmax) {
    extern __shared__ double acc[];   // [P][zmax][kb + 1]
    const int64_t K = Z.n;
    const int64_t item = blockIdx.x;
    if (item >= w.itemoff[K]) return;   // uniform over the workgroup
    const int64_t j = item_cluster(w.itemoff, K, item);
    const int64_t m0 = w.cnt[j * tiles], m1 = w.cnt[(j + 1) * tiles];
    const int64_t lo = m0 + (item - w.itemoff[j]) * kItem;
    const int64_t hi = lo + kItem < m1 ? lo + kItem : m1;
    const int64_t S = Z.off[j + 1] - Z.off[j];
    const int Sl = (int)(S < zmax ? S : zmax);   // members exist only if S <= zmax
    const int d = X.d, row = kb + 1;
    const int p = threadIdx.x / kb, c = threadIdx.x % kb;
    double *out = w.part + (size_t)item * zmax * (d + 1);
    for (int k0 = 0; k0 < d; k0 += kb) {
        for (int e = threadIdx.x; e < P * Sl * row; e += blockDim.x) acc[e] = 0.0;
        __syncthreads();
        if (p < P) {
            double *mine = acc + (size_t)p * Sl * row;
            const int k = k0 + c;
            for (int64_t m = lo + p; m < hi; m += P) {
                if (w.stm[m] != kOk) continue;
                const int64_t i = w.perm[m];
                const double om = w.objw ? w.objw[i] : 1.0;   // Eq. (4): flows weighted by the object
                const int64_t x0 = X.off[i];
                const int ncell = (int)(X.off[i + 1] - x0 + S);
                const int32_t *code = w.code + m * cs;
                const double *flow = w.flow + m * cs;
                for (int q = 0; q < ncell; q += 4) {   // four cells' loads in flight
                    int cd[4];
                    double f[4], xv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        cd[u] = q + u < ncell ? code[q + u] : -1;
                        f[u] = q + u < ncell ? flow[q + u] * om : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        xv[u] = (cd[u] >= 0 && k < d) ? ldw<TIn>(X.pts, (x0 + (cd[u] >> 16)) * d + k) : 0.0;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (cd[u] < 0) continue;
                        const int r = cd[u] & 0xffff;
                        if (k < d) mine[r * row + c] += f[u] * xv[u];
                        if (c == 0) mine[r * row + kb] += f[u];
                    }
                }
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < Sl * row; e += blockDim.x) {
            const int r = e / row, cc = e % row;
            const int k = cc < kb ? k0 + cc : d;   // column kb holds the flow total
            if (k > d || (cc < kb && k >= d)) continue;
            if (cc == kb && k0 > 0) continue;      // flow total once
            double v = 0.0;
            for (int q = 0; q < P; ++q) v += acc[((size_t)q * Sl + r) * row + cc];
            out[(size_t)r * (d + 1) + k] = v;
        }
        __syncthreads();
    }
}

// One workgroup per cluster: its items' partial rows added in item order;
// an atom with no flow keeps its coordinates.
template <typename TIn>
__global__ __launch_bounds__(256) void k_upd_finish(KSet Z, UpdWS w, int zmax, double *z_new) {
    const int64_t j = blockIdx.x;
    const int d = Z.d;
    const int64_t z0 = Z.off[j];
    const int64_t S = Z.off[j + 1] - z0;
    const int64_t Sl = S < zmax ? S : zmax;
    const int64_t it0 = w.itemoff[j], it1 = w.itemoff[j + 1];
    const size_t stride = (size_t)zmax * (d + 1);
    for (int64_t e = threadIdx.x; e < S * d; e += blockDim.x) {
        const int64_t r = e / d, k = e % d;
        const int64_t at = (z0 + r) * d + k;
        double num = 0.0, den = 0.0;
        if (r < Sl) {
            const double *src = w.part + (size_t)r * (d + 1);
            for (int64_t it = it0; it < it1; ++it) {
                num += src[it * stride + k];
                den += src[it * stride + d];
            }
        }
        z_new[at] = den > 0.0 ? num / den : ldw<TIn>(Z.pts, at);
    }
}

// ------------------------------------------------------------ Step 3

// One wave per member: lanes split into cg cell groups of kl coordinates.
template <typename TIn>
__global__ __launch_bounds__(256) void k_upd_eps(KSet X, KSet Z, UpdWS w, int64_t tiles, int cs, int kl,
                                                  const double *z_new) {
    const int64_t members = w.cnt[Z.n * tiles];
    const int lane = threadIdx.x & 63;
    const int cg = 64 / kl, grp = lane / kl, c = lane % kl;
    const int d = X.d;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t m = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; m < members; m += waves) {
        if (w.stm[m] != kOk) continue;   // uniform over the wave
        const int64_t i = w.perm[m], j = w.skey[m];
        const int64_t x0 = X.off[i], z0 = Z.off[j];
        const int ncell = (int)(X.off[i + 1] - x0 + Z.off[j + 1] - z0);
        const int32_t *code = w.code + m * cs;
        const double *flow = w.flow + m * cs;
        double e = 0.0;
        for (int q = grp; q < ncell; q += cg) {
            const int cd = code[q];
            if (cd < 0) continue;
            const int a = cd >> 16, r = cd & 0xffff;
            double part = 0.0;
            for (int k = c; k < d; k += kl) {
                const double diff = z_new[(z0 + r) * d + k] - ldw<TIn>(X.pts, (x0 + a) * d + k);
                part += diff * diff;
            }
            e += flow[q] * part;
        }
        for (int sh = 32; sh >= 1; sh >>= 1) e += __shfl_xor(e, sh, 64);
        if (lane == 0) w.eps3m[m] = e;
    }
}

// One wave per item: sums of its members' Step 1 and Step 3 values.
__global__ __launch_bounds__(256) void k_upd_isums(UpdWS w, int64_t K, int64_t tiles) {
    const int lane = threadIdx.x & 63;
    const int64_t items = w.itemoff[K];
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t item = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; item < items;
         item += waves) {
        const int64_t j = item_cluster(w.itemoff, K, item);
        const int64_t m1 = w.cnt[(j + 1) * tiles];
        const int64_t m = w.cnt[j * tiles] + (item - w.itemoff[j]) * kItem + lane;   // kItem == 64
        double a1 = 0.0, a3 = 0.0;
        int64_t cnt = 0;
        if (m < m1 && w.stm[m] == kOk) {
            const double om = w.objw ? w.objw[w.perm[m]] : 1.0;
            a1 = w.d2m[m] * om;
            a3 = w.eps3m[m] * om;
            cnt = 1;
        }
        for (int sh = 32; sh >= 1; sh >>= 1) {
            a1 += __shfl_xor(a1, sh, 64);
            a3 += __shfl_xor(a3, sh, 64);
            cnt += __shfl_xor(cnt, sh, 64);
        }
        if (lane == 0) {
            w.ie1[item] = a1;
            w.ie3[item] = a3;
            w.icnt[item] = cnt;
        }
    }
}

// One wave per cluster: its items' sums.
__global__ __launch_bounds__(256) void k_upd_csums(UpdWS w, int64_t K, double *eps1, double *eps3,
                                                    int32_t *counts) {
    const int64_t j = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    if (j >= K) return;
    const int lane = threadIdx.x & 63;
    double a1 = 0.0, a3 = 0.0;
    int64_t cnt = 0;
    for (int64_t it = w.itemoff[j] + lane; it < w.itemoff[j + 1]; it += 64) {
        a1 += w.ie1[it];
        a3 += w.ie3[it];
        cnt += w.icnt[it];
    }
    for (int sh = 32; sh >= 1; sh >>= 1) {
        a1 += __shfl_xor(a1, sh, 64);
        a3 += __shfl_xor(a3, sh, 64);
        cnt += __shfl_xor(cnt, sh, 64);
    }
    if (lane == 0) {
        if (eps1) eps1[j] = a1;
        if (eps3) eps3[j] = a3;
        if (counts) counts[j] = (int32_t)cnt;
    }
}

struct UpdSolveRun {
    const LaunchCtx &c;
    const KSet &X, &Z;
    const KOpts &o;
    int xmax, zmax;
    const UpdWS &w;
    int64_t tiles;
    int cs;
    int32_t *obj_status;
    int64_t n;
    template <int C, typename TIn, int V>
    hipError_t run() {
        const int NG = ShapeCfg<C>::groups;
        int64_t grid = (n + NG - 1) / NG;
        if (grid > (1LL << 30)) grid = 1LL << 30;
        if (grid < 1) grid = 1;
        hipLaunchKernelGGL((k_upd_solve<C, TIn, V>), dim3((unsigned)grid), dim3(ShapeCfg<C>::threads), 0,
                           c.stream, X, Z, o, xmax, zmax, w, tiles, cs, obj_status);
        return hipGetLastError();
    }
};

}  // namespace

// Coordinates per pass of the mean kernel and member slices per workgroup:
// the LDS rows (P x zmax x (kb + 1) doubles) stay within 64 KiB.
void update_mean_shape(int d, int zmax, int *kb, int *P) {
    int k = d < 64 ? d : 64;
    if (k < 1) k = 1;
    int p = 256 / k;
    const int zm = zmax > 0 ? zmax : 1;
    const int cap = (int)(65536 / ((size_t)zm * (k + 1) * 8));
    if (p > cap) p = cap;
    if (p < 1) p = 1;
    *kb = k;
    *P = p;
}

size_t update_ws_bytes(int64_t n, int64_t K, int d, int xmax, int zmax) {
    return upd_layout(upd_dims(n, K, d, xmax, zmax), nullptr, nullptr);
}

hipError_t launch_update(const LaunchCtx &c, int cls, const KSet &X, const KSet &Z, int xmax, int zmax,
                         const KOpts &o, const int32_t *labels, const double *obj_weights, double *z_new,
                         double *eps1, double *eps3, int32_t *counts, int32_t *obj_status, void *ws) {
    const UpdDims u = upd_dims(X.n, Z.n, X.d, xmax, zmax);
    UpdWS w;
    upd_layout(u, ws, &w);
    w.objw = obj_weights;
    const bool f32 = X.dtype == D2_F32;
    hipError_t e;
    const unsigned wave_blocks = (unsigned)((u.tiles + 3) / 4);   // 4 waves per block
    const int64_t fill_grid = (u.entries + 255) / 256 < 4096 ? (u.entries + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_upd_fill, dim3((unsigned)fill_grid), dim3(256), 0, c.stream, w.cnt, u.entries);
    if (X.n > 0)
        hipLaunchKernelGGL(k_upd_count, dim3(wave_blocks), dim3(256), 0, c.stream, labels, X.n, Z.n, u.tiles,
                           w.cnt, obj_status);
    hipLaunchKernelGGL(k_upd_scan_blocks, dim3((unsigned)u.sblocks), dim3(256), 0, c.stream, w.cnt, u.entries,
                       w.bsum);
    hipLaunchKernelGGL(k_upd_scan_top, dim3(1), dim3(1024), 0, c.stream, w.bsum, u.sblocks);
    hipLaunchKernelGGL(k_upd_scan_apply, dim3((unsigned)u.sblocks), dim3(256), 0, c.stream, w.cnt, u.entries,
                       w.bsum);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (X.n > 0) {
        hipLaunchKernelGGL(k_upd_place, dim3(wave_blocks), dim3(256), 0, c.stream, labels, X.n, Z.n, u.tiles,
                           w.cnt, w.perm, w.skey);
        UpdSolveRun r{c, X, Z, o, xmax, zmax, w, u.tiles, u.cs, obj_status, X.n};
        if ((e = dispatch_class(cls, f32, o.init, r)) != hipSuccess) return e;
    }
    if (Z.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_upd_items, dim3(1), dim3(1024), 0, c.stream, w.cnt, Z.n, u.tiles, w.itemoff);
    int kb, P;
    update_mean_shape(X.d, zmax, &kb, &P);
    const size_t lds = (size_t)P * zmax * (kb + 1) * sizeof(double);
    if (X.n > 0) {
        if (f32)
            hipLaunchKernelGGL(k_upd_partial<float>, dim3((unsigned)u.items), dim3(256), lds, c.stream, X, Z, w,
                               u.tiles, u.cs, kb, P, zmax);
        else
            hipLaunchKernelGGL(k_upd_partial<double>, dim3((unsigned)u.items), dim3(256), lds, c.stream, X, Z, w,
                               u.tiles, u.cs, kb, P, zmax);
    }
    if (f32)
        hipLaunchKernelGGL(k_upd_finish<float>, dim3((unsigned)Z.n), dim3(256), 0, c.stream, Z, w, zmax, z_new);
    else
        hipLaunchKernelGGL(k_upd_finish<double>, dim3((unsigned)Z.n), dim3(256), 0, c.stream, Z, w, zmax, z_new);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (X.n > 0) {
        int kl = 1;
        while (kl < X.d && kl < 64) kl <<= 1;
        const int64_t eg = (X.n + 3) / 4 < 65536 ? (X.n + 3) / 4 : 65536;
        if (f32)
            hipLaunchKernelGGL(k_upd_eps<float>, dim3((unsigned)eg), dim3(256), 0, c.stream, X, Z, w, u.tiles,
                               u.cs, kl, z_new);
        else
            hipLaunchKernelGGL(k_upd_eps<double>, dim3((unsigned)eg), dim3(256), 0, c.stream, X, Z, w, u.tiles,
                               u.cs, kl, z_new);
        const int64_t ig = (u.items + 3) / 4 < 65536 ? (u.items + 3) / 4 : 65536;
        hipLaunchKernelGGL(k_upd_isums, dim3((unsigned)ig), dim3(256), 0, c.stream, w, Z.n, u.tiles);
    }
    hipLaunchKernelGGL(k_upd_csums, dim3((unsigned)((Z.n + 3) / 4)), dim3(256), 0, c.stream, w, Z.n, eps1,
                       eps3, counts);
    return hipGetLastError();
}

}  // namespace d2
