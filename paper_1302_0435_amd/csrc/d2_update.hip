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


// ================================================= free centroid weights
//
// Alg. 1 Step 1 with the centroid weights free: for every cluster, the LP of
// Eq. (1) over the weights p_z of its s atoms and every member's matching,
// with the member's weight omega of Eq. (3) on its costs.  Members of one
// cluster are coupled through p_z, so the LP does not separate; it is solved
// whole by a revised simplex, one workgroup per cluster:
//   rows     member k's atom a (sum_r w = p_k(a)), then the coupling rows
//            sum_a w(k, ., r) - p_z(r) = 0: all s of member 0's, s - 1 of
//            each later member's (the last is implied: every member's rows
//            give sum_r p_z(r) = 1, so the mass row and one coupling row per
//            later member are dependent and dropped); m = sum t + n (s - 1) + 1;
//   columns  w(k, a, r) for every member, atom and centroid atom (two unit
//            entries), then p_z(r) (-1 in member r's coupling rows);
//   start    a basis the caller kept from an earlier pass over the same
//            members, when it still is one and is feasible; else member 0
//            sends each atom to its cheapest centroid atom, which fixes p_z
//            (all s weights basic), and every later member's transport
//            problem from its weights to p_z gets a least-cost spanning tree.
//            That basis matrix is block triangular with non-singular blocks,
//            so it is a basis;
//   pivots   explicit inverse of the basis: Dantzig's entering column
//            (Bland's after a run of degenerate pivots), the column
//            B^-1 a_q, the ratio test (least ratio, then lowest variable),
//            the rank-one update of B^-1 and of the duals y = c_B B^-1
//            (y += d_q times the new pivot row); B^-1, x_B and y are rebuilt
//            from the identity by pivoting the basis columns in, each onto
//            its largest untaken entry, every kRefactor pivots and before
//            optimality is declared; values of
//            the solution at or below kFlowEps are rounding noise of zeros
//            and set to 0;
//   Step 2   each atom moves to the omega-and-flow-weighted mean of the
//            member atoms matched to it (Eq. (4)); Step 3 evaluates the
//            objective with the moved atoms and the same matchings.
// B^-1 (m x m), the costs and the solution live in the workgroup's
// slab of the workspace, sized for the caller's bound on the members of one
// cluster; the vectors of length m and the member tables live in LDS when
// they fit in kFreeLds bytes, else in the slab.  Sums run in a fixed order.

namespace {

constexpr int kFreeThreads = 512;
constexpr int kFreeWaves = kFreeThreads / 64;
constexpr int kRefactor = 256;
constexpr double kFreeTol = 1e-13;     // reduced costs above -kFreeTol max|c| count as >= 0
constexpr double kPivTol = 1e-9;       // least entry of B^-1 a_q taken in the ratio test
constexpr double kFlowEps = 1e-14;     // flows at or below this (of a unit mass) are zeros
constexpr double kWarmTol = 1e-12;     // a kept basis starts only if B^-1 b >= -kWarmTol
// Dynamic LDS for the vectors, when they fit: a gfx950 workgroup may hold
// 160 KiB, and the kernel's registers allow one 512-thread workgroup per CU
// anyway, so nearly all of it can go to one program.
constexpr size_t kFreeLds = 150 * 1024;
enum { kFOk = 0, kFBadWeights = 1, kFTooLarge = 2, kFPivotCap = 3, kFInternal = 6 };

// Vectors of one cluster's program (length m unless noted).
struct FreeVec {
    double *y, *alpha, *xB, *prow, *b, *cB;
    double *om, *isum;    // [nmax] member weight omega, 1 / (sum of its weights)
    int64_t *obj;         // [nmax] member object
    int32_t *basis;       // variable of each basis position
    int32_t *nbasis;      // the basis being rebuilt by a reinversion
    int32_t *T;           // [nmax + 1] first row (atom) of each member
    int32_t *amem;        // [nmax xmax] member of each row (atom)
    int32_t *tt;          // [nmax] support of each member before compaction
    uint32_t *basic;      // [vmax / 32] bit v set for basic variables
    int8_t *taken;        // rows already given a basis column by a reinversion
    int16_t *rlist;       // rows a rank-one update changes (ascending)
    int16_t *clist;       // columns it changes (ascending)
};

// Byte offsets of the vectors inside their block (LDS or the slab).
struct FreeLayout {
    size_t y, alpha, xB, prow, b, cB, om, isum, obj, basis, nbasis, T, amem, tt, basic, taken, rlist, clist, total;
};

FreeLayout free_layout(int64_t nmax, int64_t amax, int64_t mmax, int64_t vmax) {
    FreeLayout l;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t q = off;
        off += (bytes + 15) & ~(size_t)15;
        return q;
    };
    l.y = take((size_t)mmax * 8);
    l.alpha = take((size_t)mmax * 8);
    l.xB = take((size_t)mmax * 8);
    l.prow = take((size_t)mmax * 8);
    l.b = take((size_t)mmax * 8);
    l.cB = take((size_t)mmax * 8);
    l.om = take((size_t)nmax * 8);
    l.isum = take((size_t)nmax * 8);
    l.obj = take((size_t)nmax * 8);
    l.basis = take((size_t)mmax * 4);
    l.nbasis = take((size_t)mmax * 4);
    l.T = take((size_t)(nmax + 1) * 4);
    l.amem = take((size_t)amax * 4);
    l.tt = take((size_t)nmax * 4);
    l.basic = take((size_t)((vmax + 31) / 32) * 4);
    l.taken = take((size_t)mmax);
    l.rlist = take((size_t)mmax * 2);
    l.clist = take((size_t)mmax * 2);
    l.total = off;
    return l;
}

__device__ __forceinline__ FreeVec free_vec(char *base, const FreeLayout &l) {
    FreeVec v;
    v.y = (double *)(base + l.y);
    v.alpha = (double *)(base + l.alpha);
    v.xB = (double *)(base + l.xB);
    v.prow = (double *)(base + l.prow);
    v.b = (double *)(base + l.b);
    v.cB = (double *)(base + l.cB);
    v.om = (double *)(base + l.om);
    v.isum = (double *)(base + l.isum);
    v.obj = (int64_t *)(base + l.obj);
    v.basis = (int32_t *)(base + l.basis);
    v.nbasis = (int32_t *)(base + l.nbasis);
    v.T = (int32_t *)(base + l.T);
    v.amem = (int32_t *)(base + l.amem);
    v.tt = (int32_t *)(base + l.tt);
    v.basic = (uint32_t *)(base + l.basic);
    v.taken = (int8_t *)(base + l.taken);
    v.rlist = (int16_t *)(base + l.rlist);
    v.clist = (int16_t *)(base + l.clist);
    return v;
}

struct FreeDims {
    int nmax, xmax, zmax, d, lds;
    int64_t mmax, vmax, amax;
    size_t vec, slab;
    FreeLayout lay;
};

FreeDims free_dims(int nmax, int xmax, int zmax, int d) {
    FreeDims f;
    f.nmax = nmax > 0 ? nmax : 1;
    f.xmax = xmax > 0 ? xmax : 1;
    f.zmax = zmax > 0 ? zmax : 1;
    f.d = d;
    f.amax = (int64_t)f.nmax * f.xmax;
    f.mmax = f.amax + (int64_t)f.nmax * (f.zmax - 1) + 1;
    f.vmax = (int64_t)f.zmax * f.amax + f.zmax;
    f.lay = free_layout(f.nmax, f.amax, f.mmax, f.vmax);
    f.vec = f.lay.total;
    f.lds = f.vec <= kFreeLds;
    f.slab = align256((size_t)f.mmax * f.mmax * 8 + (size_t)f.vmax * 8 * 2 + (f.lds ? 0 : f.vec));
    if (f.mmax > 32767) f.slab = SIZE_MAX;   // row and column lists are 16-bit
    return f;
}

struct FreeShared {
    double rv[kFreeWaves];
    int ri[kFreeWaves];
    int cr[kFreeWaves], cc[kFreeWaves];
    int n, m, stat, p, fresh, bland, warm_ok, rfail;
    double delta, dq, negx;
    long long next;   // the cluster this workgroup takes next
};

// The next slot of the launch's queue: clusters go to workgroups as they
// become free, largest member counts first, so the large programs start
// early and a workgroup that drew one takes fewer others.  Every thread of
// the workgroup calls it.
__device__ __forceinline__ int64_t free_grab(FreeShared &sh, unsigned long long *queue) {
    __syncthreads();   // every thread is done with the previous cluster's sh.next
    if (threadIdx.x == 0) sh.next = (long long)atomicAdd(queue, 1ull);
    __syncthreads();
    return (int64_t)sh.next;
}

// Queue order key of cluster j: clusters with more members first (a
// counting sort on nmax - members, stable in j); counts beyond nmax, which
// are rejected at once, go first.
__global__ void k_free_keys(const int64_t *pre, int64_t K, int64_t tiles, int nmax, int32_t *key) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < K; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t members = pre[(j + 1) * tiles] - pre[j * tiles];
        key[j] = members > nmax ? 0 : (int32_t)(nmax - members);
    }
}

// Block-wide (value, key) minimum, lowest key among equal values; keys of
// INT32_MAX are no candidates.  Every thread receives the result.
__device__ __forceinline__ void free_argmin(FreeShared &sh, double &v, int &k) {
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int ok = __shfl_xor(k, off, 64);
        if (ov < v || (ov == v && ok < k)) { v = ov; k = ok; }
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) { sh.rv[threadIdx.x >> 6] = v; sh.ri[threadIdx.x >> 6] = k; }
    __syncthreads();
    v = sh.rv[0];
    k = sh.ri[0];
    for (int q = 1; q < kFreeWaves; ++q)
        if (sh.rv[q] < v || (sh.rv[q] == v && sh.ri[q] < k)) { v = sh.rv[q]; k = sh.ri[q]; }
}

__device__ __forceinline__ double free_max(FreeShared &sh, double v) {
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh.rv[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = sh.rv[0];
    for (int q = 1; q < kFreeWaves; ++q) m = fmax(m, sh.rv[q]);
    return m;
}

// Block-wide sum in a fixed order (the same bits on every run).
__device__ __forceinline__ double free_sum(FreeShared &sh, double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh.rv[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = sh.rv[0];
    for (int q = 1; q < kFreeWaves; ++q) t += sh.rv[q];
    return t;
}

// Row of member k's coupling constraint for atom r, or -1 (dropped).
__device__ __forceinline__ int free_colrow(int sumt, int s, int k, int r) {
    if (k == 0) return sumt + r;
    if (r == s - 1) return -1;
    return sumt + s + (k - 1) * (s - 1) + r;
}

// Reduced cost of variable v under the duals y.
__device__ __forceinline__ double free_reduced(const FreeVec &V, const double *cost, int v, int n, int s,
                                               int nw, int sumt) {
    if (v < nw) {
        const int atom = v / s, r = v - atom * s;
        const int cr = free_colrow(sumt, s, V.amem[atom], r);
        return cost[v] - V.y[atom] - (cr >= 0 ? V.y[cr] : 0.0);
    }
    const int r = v - nw;
    double acc = V.y[sumt + r];   // 0 - y . a, a = -1 on every kept coupling row of atom r
    if (r < s - 1)
        for (int k = 1; k < n; ++k) acc += V.y[sumt + s + (k - 1) * (s - 1) + r];
    return acc;
}

// alpha = B^-1 a_v (thread per row).
__device__ __forceinline__ void free_ftran(const FreeVec &V, const double *Binv, int v, int m, int n, int s,
                                           int nw, int sumt) {
    if (v < nw) {
        const int atom = v / s, r = v - atom * s;
        const int cr = free_colrow(sumt, s, V.amem[atom], r);
        for (int i = threadIdx.x; i < m; i += kFreeThreads) {
            const double *row = Binv + (int64_t)i * m;
            V.alpha[i] = row[atom] + (cr >= 0 ? row[cr] : 0.0);
        }
    } else {
        const int r = v - nw;
        for (int i = threadIdx.x; i < m; i += kFreeThreads) {
            const double *row = Binv + (int64_t)i * m;
            double acc = -row[sumt + r];
            if (r < s - 1)
                for (int k = 1; k < n; ++k) acc -= row[sumt + s + (k - 1) * (s - 1) + r];
            V.alpha[i] = acc;
        }
    }
}

// B^-1 <- E B^-1 for the pivot on row pr: row pr becomes prow (the old row
// over alpha_pr), every other row i with alpha_i != 0 loses alpha_i prow;
// only the columns where prow is non-zero change.  The rows and columns
// that change are first listed in ascending order (wave ballots); then
// each wave takes kEtaRows listed rows at a time and reads kEtaCols chunks
// of 64 listed columns of them before writing any, so the loads overlap.
constexpr int kEtaRows = 4, kEtaCols = 4;
__device__ __forceinline__ void free_eta(FreeShared &sh, const FreeVec &V, double *Binv, int m, int pr) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    int nr = 0, nc = 0;
    for (int base = 0; base < m; base += kFreeThreads) {
        const int i = base + tid;
        const bool rin = i < m && (V.alpha[i] != 0.0 || i == pr);
        const bool cin = i < m && V.prow[i] != 0.0;
        const uint64_t rb = __ballot(rin), cb = __ballot(cin);
        __syncthreads();   // the previous round's counts have been read
        if (lane == 0) {
            sh.cr[wv] = __builtin_popcountll(rb);
            sh.cc[wv] = __builtin_popcountll(cb);
        }
        __syncthreads();
        int ro = nr, co = nc;
        for (int w = 0; w < kFreeWaves; ++w) {
            if (w < wv) { ro += sh.cr[w]; co += sh.cc[w]; }
            nr += sh.cr[w];
            nc += sh.cc[w];
        }
        if (rin) V.rlist[ro + __builtin_popcountll(rb & lanes_below())] = (int16_t)i;
        if (cin) V.clist[co + __builtin_popcountll(cb & lanes_below())] = (int16_t)i;
    }
    __syncthreads();
    for (int g = wv * kEtaRows; g < nr; g += kFreeWaves * kEtaRows) {
        int rows[kEtaRows];
        double als[kEtaRows];
#pragma unroll
        for (int r = 0; r < kEtaRows; ++r) {
            rows[r] = g + r < nr ? V.rlist[g + r] : -1;
            als[r] = rows[r] >= 0 ? V.alpha[rows[r]] : 0.0;
        }
        for (int c0 = 0; c0 < nc; c0 += 64 * kEtaCols) {
            int col[kEtaCols];
            double pv[kEtaCols], bv[kEtaRows][kEtaCols];
#pragma unroll
            for (int u = 0; u < kEtaCols; ++u) {
                const int jc = c0 + u * 64 + lane;
                col[u] = jc < nc ? V.clist[jc] : -1;
                pv[u] = col[u] >= 0 ? V.prow[col[u]] : 0.0;
#pragma unroll
                for (int r = 0; r < kEtaRows; ++r)
                    bv[r][u] = (col[u] >= 0 && rows[r] >= 0 && rows[r] != pr)
                                   ? Binv[(int64_t)rows[r] * m + col[u]] : 0.0;
            }
#pragma unroll
            for (int r = 0; r < kEtaRows; ++r) {
                if (rows[r] < 0) continue;
                double *row = Binv + (int64_t)rows[r] * m;
#pragma unroll
                for (int u = 0; u < kEtaCols; ++u)
                    if (col[u] >= 0) row[col[u]] = rows[r] == pr ? pv[u] : bv[r][u] - als[r] * pv[u];
            }
        }
    }
}

// Whether the current basis and its updated x_B and y already certify the
// optimum found by pricing, so that no reinversion is needed before it is
// declared: every row of the program (member rows, every coupling row,
// sum p_z = 1) holds within kCertTol for x_B scattered into x, and every
// basic variable's reduced cost is within ctol of 0, so the pricing that
// found no entering column priced with accurate duals.  x is scratch.
constexpr double kCertTol = 1e-14;
__device__ __forceinline__ bool free_certified(FreeShared &sh, const FreeVec &V, const double *cost, double *x,
                                               int m, int n, int s, int nw, int sumt, double ctol) {
    const int tid = threadIdx.x, nvar = nw + s;
    for (int v = tid; v < nvar; v += kFreeThreads) x[v] = 0.0;
    __syncthreads();
    for (int i = tid; i < m; i += kFreeThreads) x[V.basis[i]] = V.xB[i];
    __syncthreads();
    double pr = 0.0, du = 0.0;
    for (int a = tid; a < sumt; a += kFreeThreads) {
        double acc = 0.0;
        for (int r = 0; r < s; ++r) acc += x[s * a + r];
        pr = fmax(pr, fabs(acc - V.b[a]));
    }
    for (int e = tid; e < n * s; e += kFreeThreads) {
        const int k = e / s, r = e - k * s;
        double acc = 0.0;
        for (int a = V.T[k]; a < V.T[k + 1]; ++a) acc += x[s * a + r];
        pr = fmax(pr, fabs(acc - x[nw + r]));
    }
    if (tid == 0) {
        double acc = 0.0;
        for (int r = 0; r < s; ++r) acc += x[nw + r];
        pr = fmax(pr, fabs(acc - 1.0));
    }
    for (int i = tid; i < m; i += kFreeThreads) du = fmax(du, fabs(free_reduced(V, cost, V.basis[i], n, s, nw, sumt)));
    pr = free_max(sh, pr);
    du = free_max(sh, du);
    return pr <= kCertTol && du <= ctol;
}

// Orders one wavefront's global and LDS traffic between its own lanes: a
// workgroup barrier's fences without the barrier.
__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Rows up to which the first wave alone rebuilds B^-1: a column of a small
// program is a few lane steps, which the workgroup barriers of the
// many-wave rebuild would outweigh.
constexpr int kWaveRefactor = 192;
constexpr int kWaveEtaRows = 8;   // rows of a rank-one update whose loads are issued together

// The rebuild of free_refactor (same column order, pivot rule and updates)
// by wave 0, with wave-level reductions and fences in place of workgroup
// barriers; the other waves wait at the closing barrier.  Returns, in every
// thread, whether every column found a usable pivot.
__device__ __forceinline__ bool free_reinvert_wave(FreeShared &sh, const FreeVec &V, double *Binv, int m, int n,
                                                   int s, int nw) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int sumt = V.T[n];
    if (tid < 64) {
        for (int i = 0; i < m; ++i)
            for (int j = lane; j < m; j += 64) Binv[(int64_t)i * m + j] = i == j ? 1.0 : 0.0;
        for (int i = lane; i < m; i += 64) V.taken[i] = 0;
        wave_fence();
        int fail = 0;
        for (int c = 0; c < m; ++c) {
            const int v = V.basis[c];
            // alpha = B^-1 a_v, lanes over rows
            if (v < nw) {
                const int atom = v / s, r = v - atom * s;
                const int cr = free_colrow(sumt, s, V.amem[atom], r);
                for (int i = lane; i < m; i += 64) {
                    const double *row = Binv + (int64_t)i * m;
                    V.alpha[i] = row[atom] + (cr >= 0 ? row[cr] : 0.0);
                }
            } else {
                const int r = v - nw;
                for (int i = lane; i < m; i += 64) {
                    const double *row = Binv + (int64_t)i * m;
                    double acc = -row[sumt + r];
                    if (r < s - 1)
                        for (int k = 1; k < n; ++k) acc -= row[sumt + s + (k - 1) * (s - 1) + r];
                    V.alpha[i] = acc;
                }
            }
            // the untaken row of largest |alpha|, lowest on ties
            double bv = 1.0;
            int br = INT32_MAX;
            for (int i = lane; i < m; i += 64) {
                if (V.taken[i]) continue;
                const double a = -fabs(V.alpha[i]);
                if (a < bv || (a == bv && i < br)) { bv = a; br = i; }
            }
            for (int off = 32; off >= 1; off >>= 1) {
                const double ov = __shfl_xor(bv, off, 64);
                const int ok = __shfl_xor(br, off, 64);
                if (ov < bv || (ov == bv && ok < br)) { bv = ov; br = ok; }
            }
            if (!(-bv > 1e-12) || br == INT32_MAX) { fail = 1; break; }
            wave_fence();   // every lane's alpha is written
            const double ap = V.alpha[br];
            for (int j = lane; j < m; j += 64) V.prow[j] = Binv[(int64_t)br * m + j] / ap;
            wave_fence();
            // rank-one update: list the rows (alpha != 0, and br) and the
            // columns (prow != 0) in ascending order by ballots
            int nr = 0, nc = 0;
            for (int base = 0; base < m; base += 64) {
                const int i = base + lane;
                const bool rin = i < m && (V.alpha[i] != 0.0 || i == br);
                const bool cin = i < m && V.prow[i] != 0.0;
                const uint64_t rb = __ballot(rin), cb = __ballot(cin);
                if (rin) V.rlist[nr + __builtin_popcountll(rb & lanes_below())] = (int16_t)i;
                if (cin) V.clist[nc + __builtin_popcountll(cb & lanes_below())] = (int16_t)i;
                nr += __builtin_popcountll(rb);
                nc += __builtin_popcountll(cb);
            }
            wave_fence();
            for (int g = 0; g < nr; g += kWaveEtaRows) {
                int rows[kWaveEtaRows];
                double als[kWaveEtaRows];
#pragma unroll
                for (int q = 0; q < kWaveEtaRows; ++q) {
                    rows[q] = g + q < nr ? V.rlist[g + q] : -1;
                    als[q] = rows[q] >= 0 ? V.alpha[rows[q]] : 0.0;
                }
                for (int c0 = 0; c0 < nc; c0 += 64) {
                    const int jc = c0 + lane;
                    const int col = jc < nc ? V.clist[jc] : -1;
                    const double pv = col >= 0 ? V.prow[col] : 0.0;
                    double bvals[kWaveEtaRows];
#pragma unroll
                    for (int q = 0; q < kWaveEtaRows; ++q)
                        bvals[q] = (col >= 0 && rows[q] >= 0 && rows[q] != br) ? Binv[(int64_t)rows[q] * m + col] : 0.0;
#pragma unroll
                    for (int q = 0; q < kWaveEtaRows; ++q)
                        if (col >= 0 && rows[q] >= 0)
                            Binv[(int64_t)rows[q] * m + col] = rows[q] == br ? pv : bvals[q] - als[q] * pv;
                }
            }
            if (lane == 0) {
                V.taken[br] = 1;
                V.nbasis[br] = v;
            }
            wave_fence();
        }
        if (lane == 0) sh.rfail = fail;
    }
    __syncthreads();
    return sh.rfail == 0;
}

// Rebuild B^-1 from the basis by pivoting its columns in, one by one, from
// the identity (each onto the untaken row of largest |entry|, the lowest on
// ties), then x_B = B^-1 b, c_B and y = c_B B^-1.  Returns false when a
// column has no usable pivot (the basis lost rank numerically).
__device__ __forceinline__ bool free_refactor(FreeShared &sh, const FreeVec &V, double *Binv, const double *cost,
                                              int m, int n, int s, int nw) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int sumt = V.T[n];
    const bool small = m <= kWaveRefactor;
    if (small && !free_reinvert_wave(sh, V, Binv, m, n, s, nw)) return false;
    for (int i = wv; i < m && !small; i += kFreeWaves)
        for (int j = lane; j < m; j += 64) Binv[(int64_t)i * m + j] = i == j ? 1.0 : 0.0;
    for (int i = tid; i < m && !small; i += kFreeThreads) V.taken[i] = 0;
    __syncthreads();
    for (int c = 0; c < m && !small; ++c) {
        const int v = V.basis[c];
        // each thread reads back only its own rows of alpha before the
        // reduction's barriers, so none is needed here
        free_ftran(V, Binv, v, m, n, s, nw, sumt);
        double bv = 1.0;
        int br = INT32_MAX;
        for (int i = tid; i < m; i += kFreeThreads) {
            if (V.taken[i]) continue;
            const double a = -fabs(V.alpha[i]);
            if (a < bv || (a == bv && i < br)) { bv = a; br = i; }
        }
        free_argmin(sh, bv, br);
        if (!(-bv > 1e-12) || br == INT32_MAX) return false;
        const double ap = V.alpha[br];
        // free_eta lists its own entries first and updates B^-1 only after
        // its barriers, so row br is read here before any thread writes it
        for (int j = tid; j < m; j += kFreeThreads) V.prow[j] = Binv[(int64_t)br * m + j] / ap;
        free_eta(sh, V, Binv, m, br);
        if (tid == 0) {
            V.taken[br] = 1;
            V.nbasis[br] = v;
        }
        __syncthreads();
    }
    double neg = 0.0;
    for (int i = tid; i < m; i += kFreeThreads) {
        V.basis[i] = V.nbasis[i];
        V.cB[i] = cost[V.nbasis[i]];
        double acc = 0.0;
        const double *row = Binv + (int64_t)i * m;
        for (int j = 0; j < m; ++j) acc = fma(row[j], V.b[j], acc);
        V.xB[i] = acc < 0.0 ? 0.0 : acc;
        neg = fmax(neg, -acc);
    }
    neg = free_max(sh, neg);   // the most negative basic value, before clamping
    if (tid == 0) sh.negx = neg;
    __syncthreads();
    for (int i = tid; i < m; i += kFreeThreads) {
        double acc = 0.0;
        for (int j = 0; j < m; ++j) acc = fma(V.cB[j], Binv[(int64_t)j * m + i], acc);
        V.y[i] = acc;
    }
    __syncthreads();
    return true;
}

template <typename TIn, bool L>
__global__ __launch_bounds__(kFreeThreads) void k_free_solve(KSet X, KSet Z, KOpts o, const int64_t *pre,
                                                             const int64_t *perm, int64_t tiles, FreeDims f,
                                                             char *slabs, const double *objw, double *z_new,
                                                             double *w_new, double *eps1, double *eps3,
                                                             int32_t *counts, int32_t *obj_status,
                                                             int32_t *cluster_status, int32_t *cluster_pivots,
                                                             int32_t *basis_io, int64_t bstride,
                                                             unsigned long long *queue, const int64_t *order) {
    extern __shared__ __align__(16) char free_lds[];
    __shared__ FreeShared sh;
    const int tid = threadIdx.x;
    double *Binv = (double *)(slabs + (size_t)blockIdx.x * f.slab);
    double *cost = Binv + f.mmax * f.mmax;
    double *x = cost + f.vmax;
    const FreeVec V = free_vec(L ? free_lds : (char *)(x + f.vmax), f.lay);
    const int d = X.d;
    for (int64_t slot = free_grab(sh, queue); slot < Z.n; slot = free_grab(sh, queue)) {
        const int64_t j = order[slot];
        const int64_t pb = pre[j * tiles], pe = pre[(j + 1) * tiles];
        const int64_t z0 = Z.off[j];
        const int s = (int)(Z.off[j + 1] - z0);
        // centroid outputs default to the input (kept when the LP is not solved)
        for (int64_t e = tid; e < (int64_t)s * d; e += kFreeThreads)
            z_new[z0 * d + e] = ldw<TIn>(Z.pts, z0 * d + e);
        for (int r = tid; r < s; r += kFreeThreads) w_new[z0 + r] = ldw<TIn>(Z.w, z0 + r);
        const int64_t nall = pe - pb;
        if (nall > f.nmax || s < 1 || s > f.zmax) {
            for (int64_t q = pb + tid; q < pe; q += kFreeThreads)
                if (obj_status) obj_status[perm[q]] = kFTooLarge;
            if (tid == 0) {
                if (eps1) eps1[j] = __builtin_nan("");
                if (eps3) eps3[j] = __builtin_nan("");
                if (counts) counts[j] = 0;
                if (cluster_status) cluster_status[j] = kFTooLarge;
                if (cluster_pivots) cluster_pivots[j] = 0;
                if (basis_io) basis_io[j * bstride] = -1;
            }
            __syncthreads();
            continue;
        }
        // members: validate (thread per member), then compact in order
        for (int64_t q = pb + tid; q < pe; q += kFreeThreads) {
            const int64_t i = perm[q];
            const int64_t a0 = X.off[i];
            const int64_t t = X.off[i + 1] - a0;
            const double om = objw ? objw[i] : 1.0;
            double sum = 0.0;
            bool bad = !(isfinite(om) && om >= 0.0) || t < 1 || t > f.xmax;
            for (int64_t a = 0; a < t && !bad; ++a) {
                const double w = ldw<TIn>(X.w, a0 + a);
                bad = !(isfinite(w) && w >= 0.0);
                sum += w;
            }
            bad = bad || !(sum > 0.0) || !isfinite(sum);
            if (obj_status) obj_status[i] = bad ? (t > f.xmax ? kFTooLarge : kFBadWeights) : kFOk;
            V.isum[q - pb] = bad ? -1.0 : (om > 0.0 ? 1.0 / sum : 0.0);
            V.om[q - pb] = om;
            V.obj[q - pb] = i;
            V.tt[q - pb] = (int)t;
        }
        __syncthreads();
        if (tid == 0) {
            int n = 0, acc = 0;
            for (int q = 0; q < (int)nall; ++q) {
                if (!(V.isum[q] > 0.0)) continue;   // invalid, or omega = 0: no part in the LP
                V.obj[n] = V.obj[q];
                V.om[n] = V.om[q];
                V.isum[n] = V.isum[q];
                V.T[n] = acc;
                acc += V.tt[q];
                ++n;
            }
            V.T[n] = acc;
            sh.n = n;
            sh.m = acc + n * (s - 1) + 1;
            sh.stat = kFOk;
        }
        __syncthreads();
        const int n = sh.n, m = sh.m, sumt = V.T[n], nw = s * sumt, nvar = nw + s;
        if (n == 0) {
            if (tid == 0) {
                if (eps1) eps1[j] = 0.0;
                if (eps3) eps3[j] = 0.0;
                if (counts) counts[j] = 0;
                if (cluster_status) cluster_status[j] = kFOk;
                if (cluster_pivots) cluster_pivots[j] = 0;
                if (basis_io) basis_io[j * bstride] = -1;
            }
            __syncthreads();
            continue;
        }
        // row tables and right-hand sides: the members' normalised weights, then zeros
        for (int k = tid; k < n; k += kFreeThreads) {
            const int64_t xa = X.off[V.obj[k]];
            for (int a = V.T[k]; a < V.T[k + 1]; ++a) {
                V.amem[a] = k;
                V.b[a] = ldw<TIn>(X.w, xa + (a - V.T[k])) * V.isum[k];
            }
        }
        for (int i = sumt + tid; i < m; i += kFreeThreads) V.b[i] = 0.0;
        __syncthreads();
        // costs omega_k |z_r - v_ka|^2 (direct form, coordinates ascending)
        double cm = 0.0;
        for (int v = tid; v < nvar; v += kFreeThreads) {
            double c = 0.0;
            if (v < nw) {
                const int atom = v / s, r = v - atom * s, k = V.amem[atom];
                const int64_t xa = (X.off[V.obj[k]] + (atom - V.T[k])) * d, zr = (z0 + r) * d;
                double acc = 0.0;
                for (int qd = 0; qd < d; ++qd) {
                    const double diff = ldw<TIn>(X.pts, xa + qd) - ldw<TIn>(Z.pts, zr + qd);
                    acc = fma(diff, diff, acc);
                }
                c = V.om[k] * acc;
            }
            cost[v] = c;
            cm = fmax(cm, fabs(c));
        }
        for (int w = tid; w < (nvar + 31) / 32; w += kFreeThreads) V.basic[w] = 0u;
        cm = free_max(sh, cm);
        // a kept basis of this size (an earlier pass over the same members,
        // with other atom positions) starts the simplex when its variables
        // are distinct and in range, it has full rank and its solution is
        // feasible; otherwise the structured start below
        bool warm = false;
        if (basis_io && (int64_t)m + 1 <= bstride && basis_io[j * bstride] == m) {
            const int32_t *kept = basis_io + j * bstride + 1;
            for (int i = tid; i < m; i += kFreeThreads) V.basis[i] = kept[i];
            __syncthreads();
            if (tid == 0) {
                int ok = 1;
                for (int q = 0; q < m && ok; ++q) {
                    const int v = V.basis[q];
                    if (v < 0 || v >= nvar || ((V.basic[v >> 5] >> (v & 31)) & 1u)) ok = 0;
                    else V.basic[v >> 5] |= 1u << (v & 31);
                }
                sh.warm_ok = ok;
                sh.delta = kFreeTol * cm;
                sh.fresh = 1;
                sh.bland = 0;
                sh.stat = kFOk;
            }
            __syncthreads();
            if (sh.warm_ok && free_refactor(sh, V, Binv, cost, m, n, s, nw) && !(sh.negx > kWarmTol)) warm = true;
            __syncthreads();
            if (!warm)
                for (int w = tid; w < (nvar + 31) / 32; w += kFreeThreads) V.basic[w] = 0u;
            __syncthreads();
        }
        // the structured starting basis: member 0's atoms at their cheapest
        // centroid atom (lowest on ties), thread per atom, and the weights p_z
        // they fix; then every later member's transport problem from its
        // weights to p_z by the least-cost rule, thread per member
        const int t0 = V.T[1];
        for (int a = tid; a < t0 && !warm; a += kFreeThreads) {
            int rb = 0;
            for (int r = 1; r < s; ++r)
                if (cost[a * s + r] < cost[a * s + rb]) rb = r;
            V.basis[a] = a * s + rb;
        }
        __syncthreads();
        double *pz = V.prow;   // scratch until the reinversion: the weights member 0 fixes
        if (tid == 0 && !warm) {
            sh.delta = kFreeTol * cm;
            for (int r = 0; r < s; ++r) pz[r] = 0.0;
            for (int a = 0; a < t0; ++a) pz[V.basis[a] - a * s] += V.b[a];
            for (int r = 0; r < s; ++r) V.basis[t0 + r] = nw + r;
            sh.stat = kFOk;
        }
        __syncthreads();
        // Least cost: the cheapest cell of an open row and an open column
        // (lowest row, then column, on ties) takes all that its row or column
        // has left and closes the row when the row runs out first or both do
        // (unless it is the last open row), else the column.  Each cell
        // closes a line, so the t + s - 1 cells hold no cycle: a spanning
        // tree, like the north-west corner's, and the basis stays block
        // triangular with non-singular blocks.  Remaining masses go to
        // alpha (rows) and x_B (member k's columns at (k - 1) s), both free
        // until the reinversion.
        for (int k = 1 + tid; k < n && !warm; k += kFreeThreads) {
            const int r0 = V.T[k], tk = V.T[k + 1] - r0;
            double *remr = V.alpha + r0, *remc = V.xB + (int64_t)(k - 1) * s;
            for (int a = 0; a < tk; ++a) remr[a] = V.b[r0 + a];
            for (int r = 0; r < s; ++r) remc[r] = pz[r];
            uint64_t ron = tk == 64 ? ~0ull : (1ull << tk) - 1ull;
            uint64_t con = s == 64 ? ~0ull : (1ull << s) - 1ull;
            int nb = t0 + s + (r0 - t0) + (k - 1) * (s - 1);
            for (int cell = 0; cell < tk + s - 1; ++cell) {
                double best = INFINITY;
                int ba = -1, br = -1;
                for (uint64_t ra = ron; ra; ra &= ra - 1) {
                    const int a = __builtin_ctzll(ra);
                    const double *crow = cost + (int64_t)s * (r0 + a);
                    for (uint64_t rc = con; rc; rc &= rc - 1) {
                        const int r = __builtin_ctzll(rc);
                        if (crow[r] < best || ba < 0) { best = crow[r]; ba = a; br = r; }
                    }
                }
                if (ba < 0) { sh.stat = kFInternal; break; }
                V.basis[nb++] = s * (r0 + ba) + br;
                const double fl = fmin(remr[ba], remc[br]);
                remr[ba] -= fl;
                remc[br] -= fl;
                if ((remr[ba] <= remc[br] && __popcll(ron) > 1) || __popcll(con) == 1) ron &= ~(1ull << ba);
                else con &= ~(1ull << br);
            }
        }
        __syncthreads();
        if (tid == 0 && !warm && sh.stat == kFOk) {
            for (int q = 0; q < m; ++q) V.basic[V.basis[q] >> 5] |= 1u << (V.basis[q] & 31);
            sh.fresh = 1;
            sh.bland = 0;
        }
        __syncthreads();
        if (!warm && sh.stat == kFOk && !free_refactor(sh, V, Binv, cost, m, n, s, nw) && tid == 0)
            sh.stat = kFInternal;
        __syncthreads();
        // the simplex
        const int64_t cap = o.max_pivots > 0 ? o.max_pivots : (50LL * m > 100 ? 50LL * m : 100LL);
        const int bland_after = o.bland_after > 0 ? o.bland_after : 2 * m;
        const double delta = sh.delta;
        int64_t pivots = 0;
        int streak = 0, since = 0;
        while (sh.stat == kFOk) {
            // pricing: Dantzig (least reduced cost, lowest variable), or
            // Bland (lowest variable below -delta)
            const bool bl = sh.bland != 0;
            double bv = INFINITY;
            int bq = INT32_MAX;
            for (int v = tid; v < nvar; v += kFreeThreads) {
                if ((V.basic[v >> 5] >> (v & 31)) & 1u) continue;
                const double dv = free_reduced(V, cost, v, n, s, nw, sumt);
                if (!(dv < -delta)) continue;
                const double key = bl ? 0.0 : dv;
                if (key < bv || (key == bv && v < bq)) { bv = key; bq = v; }
            }
            free_argmin(sh, bv, bq);
            if (bq == INT32_MAX) {
                if (sh.fresh) break;   // optimal with a freshly rebuilt B^-1
                // or with an updated one whose vertex and duals check out
                if (free_certified(sh, V, cost, x, m, n, s, nw, sumt, 1e-2 * delta)) break;
                __syncthreads();
                if (!free_refactor(sh, V, Binv, cost, m, n, s, nw)) {
                    if (tid == 0) sh.stat = kFInternal;
                    __syncthreads();
                    break;
                }
                if (tid == 0) sh.fresh = 1;
                since = 0;
                __syncthreads();
                continue;
            }
            if (pivots >= cap) { if (tid == 0) sh.stat = kFPivotCap; __syncthreads(); break; }
            // alpha = B^-1 a_q, and d_q
            const int q = bq;
            if (tid == 0) sh.dq = free_reduced(V, cost, q, n, s, nw, sumt);
            free_ftran(V, Binv, q, m, n, s, nw, sumt);   // own rows only until the next barrier
            // ratio test: least x_B / alpha over alpha > kPivTol, then lowest
            // variable; the winning thread names the row
            double tv = INFINITY;
            int tk = INT32_MAX, ti = -1;
            for (int i = tid; i < m; i += kFreeThreads) {
                const double al = V.alpha[i];
                if (al > kPivTol) {
                    const double r = V.xB[i] / al;
                    const int key = V.basis[i];
                    if (r < tv || (r == tv && key < tk)) { tv = r; tk = key; ti = i; }
                }
            }
            const int my_k = tk, my_i = ti;
            free_argmin(sh, tv, tk);
            if (tk == INT32_MAX) { if (tid == 0) sh.stat = kFInternal; __syncthreads(); break; }
            if (my_k == tk) sh.p = my_i;
            __syncthreads();
            const int pr = sh.p;
            const double theta = tv > 0.0 ? tv : 0.0, ap = V.alpha[pr], dq = sh.dq;
            for (int jj = tid; jj < m; jj += kFreeThreads) V.prow[jj] = Binv[(int64_t)pr * m + jj] / ap;
            free_eta(sh, V, Binv, m, pr);   // barriers before it writes B^-1 or reads others' entries
            for (int i = tid; i < m; i += kFreeThreads) {
                const double xv = i == pr ? theta : V.xB[i] - theta * V.alpha[i];
                V.xB[i] = xv < 0.0 ? 0.0 : xv;
                V.y[i] = fma(dq, V.prow[i], V.y[i]);
            }
            __syncthreads();
            if (tid == 0) {
                V.basic[V.basis[pr] >> 5] &= ~(1u << (V.basis[pr] & 31));
                V.basic[q >> 5] |= 1u << (q & 31);
                V.basis[pr] = q;
                V.cB[pr] = cost[q];
                sh.fresh = 0;
                if (theta == 0.0) {
                    if (++streak >= bland_after) sh.bland = 1;
                } else {
                    streak = 0;
                    sh.bland = 0;
                }
            }
            ++pivots;
            if (++since >= kRefactor) {
                __syncthreads();
                if (!free_refactor(sh, V, Binv, cost, m, n, s, nw)) {
                    if (tid == 0) sh.stat = kFInternal;
                    __syncthreads();
                    break;
                }
                if (tid == 0) sh.fresh = 1;
                since = 0;
            }
            __syncthreads();
        }
        __syncthreads();
        const int st = sh.stat;
        if (st != kFOk) {
            for (int k = tid; k < n; k += kFreeThreads)
                if (obj_status) obj_status[V.obj[k]] = st;
            if (tid == 0) {
                if (eps1) eps1[j] = __builtin_nan("");
                if (eps3) eps3[j] = __builtin_nan("");
                if (counts) counts[j] = 0;
                if (cluster_status) cluster_status[j] = st;
                if (cluster_pivots) cluster_pivots[j] = (int32_t)pivots;
                if (basis_io) basis_io[j * bstride] = -1;
            }
            __syncthreads();
            continue;
        }
        // the optimal basis, for a later pass's start
        if (basis_io) {
            const bool fits = (int64_t)m + 1 <= bstride;
            for (int i = tid; i < m && fits; i += kFreeThreads) basis_io[j * bstride + 1 + i] = V.basis[i];
            if (tid == 0) basis_io[j * bstride] = fits ? m : -1;
        }
        // the solution, densely
        for (int v = tid; v < nvar; v += kFreeThreads) x[v] = 0.0;
        __syncthreads();
        for (int i = tid; i < m; i += kFreeThreads) x[V.basis[i]] = V.xB[i] > kFlowEps ? V.xB[i] : 0.0;
        __syncthreads();
        for (int r = tid; r < s; r += kFreeThreads) w_new[z0 + r] = x[nw + r];
        // Step 1 value
        double p1 = 0.0;
        for (int v = tid; v < nw; v += kFreeThreads) p1 = fma(cost[v], x[v], p1);
        const double v1 = free_sum(sh, p1);
        // Step 2: each atom to the omega-and-flow-weighted mean (Eq. (4)),
        // members and atoms in order; an atom with no mass stays
        for (int e = tid; e < s * d; e += kFreeThreads) {
            const int r = e / d, qd = e - r * d;
            double num = 0.0, den = 0.0;
            for (int k = 0; k < n; ++k) {
                const int64_t xa = X.off[V.obj[k]];
                double nk = 0.0, dk = 0.0;
                for (int a = V.T[k]; a < V.T[k + 1]; ++a) {
                    const double wv2 = x[s * a + r];
                    nk = fma(wv2, ldw<TIn>(X.pts, (xa + (a - V.T[k])) * d + qd), nk);
                    dk += wv2;
                }
                num = fma(V.om[k], nk, num);
                den = fma(V.om[k], dk, den);
            }
            if (den > 0.0) z_new[(z0 + r) * d + qd] = num / den;
        }
        __syncthreads();
        // Step 3: the objective with the moved atoms and the same matchings
        double p3 = 0.0;
        for (int v = tid; v < nw; v += kFreeThreads) {
            const double wv2 = x[v];
            if (wv2 == 0.0) continue;
            const int atom = v / s, r = v - atom * s, k = V.amem[atom];
            const int64_t xa = (X.off[V.obj[k]] + (atom - V.T[k])) * d;
            double acc = 0.0;
            for (int qd = 0; qd < d; ++qd) {
                const double diff = ldw<TIn>(X.pts, xa + qd) - z_new[(z0 + r) * d + qd];
                acc = fma(diff, diff, acc);
            }
            p3 = fma(V.om[k] * wv2, acc, p3);
        }
        const double v3 = free_sum(sh, p3);
        if (tid == 0) {
            if (eps1) eps1[j] = v1;
            if (eps3) eps3[j] = v3;
            if (counts) counts[j] = n;
            if (cluster_status) cluster_status[j] = kFOk;
            if (cluster_pivots) cluster_pivots[j] = (int32_t)pivots;
        }
        __syncthreads();
    }
}

}  // namespace

// Workspace of the clusters' queue order (a counting sort of K clusters
// over nmax + 1 keys).
size_t free_queue_bytes(int64_t K, int nmax) {
    const UpdDims q = upd_dims(K, (int64_t)nmax + 1, 1, 1, 1);
    const int64_t k1 = K > 0 ? K : 1;
    return align256((size_t)k1 * 4) + align256((size_t)q.entries * 8) + align256((size_t)q.sblocks * 8) +
           align256((size_t)k1 * 8) + align256((size_t)k1 * 4);
}

size_t update_free_slab_bytes(int max_members, int xmax, int zmax, int d) {
    return free_dims(max_members, xmax, zmax, d).slab;
}

size_t update_free_ws_bytes(int64_t n, int64_t K, int d, int xmax, int zmax, int max_members, int cu_count,
                            int64_t *grid_out) {
    const UpdDims u = upd_dims(n, K, d, xmax, zmax);
    const FreeDims f = free_dims(max_members, xmax, zmax, d);
    // two workgroups per CU, the slabs within 4 GiB
    int64_t grid = (int64_t)(cu_count > 0 ? cu_count : 256) * 2;
    const int64_t fit = (int64_t)(((size_t)4 << 30) / f.slab);
    if (grid > fit) grid = fit;
    if (grid > K) grid = K;
    if (grid < 1) grid = 1;
    if (grid_out) *grid_out = grid;
    // grouping arrays (counts, block sums, order, keys), the queue counter
    // and the clusters' queue order (keys, counts, block sums, order,
    // sorted keys), then the slabs
    return align256((size_t)u.entries * 8) + align256((size_t)u.sblocks * 8) + align256((size_t)(n > 0 ? n : 1) * 8) +
           align256((size_t)(n > 0 ? n : 1) * 4) + align256(8) + free_queue_bytes(K, f.nmax) + (size_t)grid * f.slab;
}

hipError_t launch_update_free(const LaunchCtx &c, const KSet &X, const KSet &Z, int xmax, int zmax,
                              int max_members, const KOpts &o, const int32_t *labels, const double *obj_weights,
                              double *z_new, double *w_new, double *eps1, double *eps3, int32_t *counts,
                              int32_t *obj_status, int32_t *cluster_status, int32_t *cluster_pivots,
                              int32_t *basis_io, int64_t basis_stride, void *ws) {
    const UpdDims u = upd_dims(X.n, Z.n, X.d, xmax, zmax);
    const FreeDims f = free_dims(max_members, xmax, zmax, X.d);
    int64_t grid = 1;
    update_free_ws_bytes(X.n, Z.n, X.d, xmax, zmax, max_members, c.cu_count, &grid);
    char *p = (char *)ws;
    int64_t *cnt = (int64_t *)p;
    p += align256((size_t)u.entries * 8);
    int64_t *bsum = (int64_t *)p;
    p += align256((size_t)u.sblocks * 8);
    int64_t *perm = (int64_t *)p;
    p += align256((size_t)(X.n > 0 ? X.n : 1) * 8);
    int32_t *skey = (int32_t *)p;
    p += align256((size_t)(X.n > 0 ? X.n : 1) * 4);
    unsigned long long *queue = (unsigned long long *)p;
    p += align256(8);
    const UpdDims q = upd_dims(Z.n, (int64_t)f.nmax + 1, 1, 1, 1);
    const int64_t k1 = Z.n > 0 ? Z.n : 1;
    int32_t *qkey = (int32_t *)p;
    p += align256((size_t)k1 * 4);
    int64_t *qcnt = (int64_t *)p;
    p += align256((size_t)q.entries * 8);
    int64_t *qbsum = (int64_t *)p;
    p += align256((size_t)q.sblocks * 8);
    int64_t *order = (int64_t *)p;
    p += align256((size_t)k1 * 8);
    int32_t *qskey = (int32_t *)p;
    p += align256((size_t)k1 * 4);
    char *slabs = p;
    const unsigned wave_blocks = (unsigned)((u.tiles + 3) / 4);
    const int64_t fill_grid = (u.entries + 255) / 256 < 4096 ? (u.entries + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_upd_fill, dim3((unsigned)fill_grid), dim3(256), 0, c.stream, cnt, u.entries);
    hipLaunchKernelGGL(k_upd_fill, dim3(1), dim3(64), 0, c.stream, (int64_t *)queue, (int64_t)1);
    if (X.n > 0)
        hipLaunchKernelGGL(k_upd_count, dim3(wave_blocks), dim3(256), 0, c.stream, labels, X.n, Z.n, u.tiles, cnt,
                           obj_status);
    hipLaunchKernelGGL(k_upd_scan_blocks, dim3((unsigned)u.sblocks), dim3(256), 0, c.stream, cnt, u.entries, bsum);
    hipLaunchKernelGGL(k_upd_scan_top, dim3(1), dim3(1024), 0, c.stream, bsum, u.sblocks);
    hipLaunchKernelGGL(k_upd_scan_apply, dim3((unsigned)u.sblocks), dim3(256), 0, c.stream, cnt, u.entries, bsum);
    if (X.n > 0)
        hipLaunchKernelGGL(k_upd_place, dim3(wave_blocks), dim3(256), 0, c.stream, labels, X.n, Z.n, u.tiles, cnt,
                           perm, skey);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || Z.n == 0) return e;
    // the queue order: clusters by member count, largest first
    {
        const unsigned kb = (unsigned)((Z.n + 255) / 256 < 4096 ? (Z.n + 255) / 256 : 4096);
        hipLaunchKernelGGL(k_free_keys, dim3(kb), dim3(256), 0, c.stream, cnt, Z.n, u.tiles, f.nmax, qkey);
        const int64_t qfill = (q.entries + 255) / 256 < 4096 ? (q.entries + 255) / 256 : 4096;
        const unsigned qwave = (unsigned)((q.tiles + 3) / 4);
        hipLaunchKernelGGL(k_upd_fill, dim3((unsigned)qfill), dim3(256), 0, c.stream, qcnt, q.entries);
        hipLaunchKernelGGL(k_upd_count, dim3(qwave), dim3(256), 0, c.stream, qkey, Z.n, q.K, q.tiles, qcnt,
                           (int32_t *)nullptr);
        hipLaunchKernelGGL(k_upd_scan_blocks, dim3((unsigned)q.sblocks), dim3(256), 0, c.stream, qcnt, q.entries,
                           qbsum);
        hipLaunchKernelGGL(k_upd_scan_top, dim3(1), dim3(1024), 0, c.stream, qbsum, q.sblocks);
        hipLaunchKernelGGL(k_upd_scan_apply, dim3((unsigned)q.sblocks), dim3(256), 0, c.stream, qcnt, q.entries,
                           qbsum);
        hipLaunchKernelGGL(k_upd_place, dim3(qwave), dim3(256), 0, c.stream, qkey, Z.n, q.K, q.tiles, qcnt, order,
                           qskey);
    }
    const size_t lds = f.lds ? f.vec : 0;
    if (X.dtype == D2_F32) {
        if (f.lds)
            hipLaunchKernelGGL((k_free_solve<float, true>), dim3((unsigned)grid), dim3(kFreeThreads), lds, c.stream,
                               X, Z, o, cnt, perm, u.tiles, f, slabs, obj_weights, z_new, w_new, eps1, eps3, counts,
                               obj_status, cluster_status, cluster_pivots, basis_io, basis_stride, queue, order);
        else
            hipLaunchKernelGGL((k_free_solve<float, false>), dim3((unsigned)grid), dim3(kFreeThreads), 0, c.stream,
                               X, Z, o, cnt, perm, u.tiles, f, slabs, obj_weights, z_new, w_new, eps1, eps3, counts,
                               obj_status, cluster_status, cluster_pivots, basis_io, basis_stride, queue, order);
    } else {
        if (f.lds)
            hipLaunchKernelGGL((k_free_solve<double, true>), dim3((unsigned)grid), dim3(kFreeThreads), lds, c.stream,
                               X, Z, o, cnt, perm, u.tiles, f, slabs, obj_weights, z_new, w_new, eps1, eps3, counts,
                               obj_status, cluster_status, cluster_pivots, basis_io, basis_stride, queue, order);
        else
            hipLaunchKernelGGL((k_free_solve<double, false>), dim3((unsigned)grid), dim3(kFreeThreads), 0, c.stream,
                               X, Z, o, cnt, perm, u.tiles, f, slabs, obj_weights, z_new, w_new, eps1, eps3, counts,
                               obj_status, cluster_status, cluster_pivots, basis_io, basis_stride, queue, order);
    }
    return hipGetLastError();
}

// ================================================= merging a level
//
// Alg. 3 Step 3 for one level (Sec. 2.4): the centroids with members are
// kept and renumbered in order (the segments' centroid ranges are
// consecutive, so this is the offset of Eq. (5)), each kept centroid's
// weight is the sum of its members' weights (Eq. (3)), its atoms are copied
// into the next level's object set, and every original object inherits the
// new label of its level object (Eq. (6)).  Members are grouped by the same
// counting sort as the update, so the weight sums run in member order.

namespace {

// new_index[j] = kept centroids before j (j = 0..K; new_index[K] = the kept
// count), then the kept centroids' atom offsets in their new order.
__global__ __launch_bounds__(1024) void k_merge_index(const int64_t *pre, int64_t K, int64_t tiles,
                                                       const int64_t *zoff, int64_t *new_index, int64_t *new_off,
                                                       int64_t *kept) {
    for (int64_t j = threadIdx.x; j <= K; j += blockDim.x)
        new_index[j] = (j < K && pre[(j + 1) * tiles] > pre[j * tiles]) ? 1 : 0;
    __syncthreads();
    block_exclusive_scan(new_index, K + 1);
    __syncthreads();
    const int64_t q = new_index[K];
    for (int64_t j = threadIdx.x; j < K; j += blockDim.x)
        if (pre[(j + 1) * tiles] > pre[j * tiles]) new_off[new_index[j]] = zoff[j + 1] - zoff[j];
    if (threadIdx.x == 0) new_off[q] = 0;
    __syncthreads();
    block_exclusive_scan(new_off, q + 1);
    if (threadIdx.x == 0) *kept = q;
}

// Kept centroid weights: its members' weights summed in member order.
__global__ void k_merge_weights(const int64_t *pre, const int64_t *perm, int64_t K, int64_t tiles,
                                const double *omega, const int64_t *new_index, double *new_omega) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < K; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = pre[j * tiles], e = pre[(j + 1) * tiles];
        if (e <= b) continue;
        double sum = 0.0;
        for (int64_t q = b; q < e; ++q) sum += omega ? omega[perm[q]] : 1.0;
        new_omega[new_index[j]] = sum;
    }
}

// Atoms of the kept centroids, in their new order (one wave per centroid).
template <typename T>
__global__ void k_merge_gather(const int64_t *zoff, const T *zpts, const T *zw, int d, int64_t K,
                               const int64_t *pre, int64_t tiles, const int64_t *new_index,
                               const int64_t *new_off, T *npts, T *nw) {
    const int lane = threadIdx.x & 63;
    for (int64_t j = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; j < K;
         j += (int64_t)gridDim.x * (blockDim.x / 64)) {
        if (pre[(j + 1) * tiles] <= pre[j * tiles]) continue;
        const int64_t src = zoff[j], dst = new_off[new_index[j]], s = zoff[j + 1] - zoff[j];
        for (int64_t e = lane; e < s * d; e += 64) npts[dst * d + e] = zpts[src * d + e];
        for (int64_t a = lane; a < s; a += 64) nw[dst + a] = zw[src + a];
    }
}

// Eq. (6): an original object's new label is that of its level object.
__global__ void k_merge_inherit(const int32_t *labels, int64_t n, int64_t K, const int64_t *new_index, int32_t *C,
                                int64_t n0) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n0; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = C[i];
        const int32_t lab = (c >= 0 && c < n) ? labels[c] : -1;
        C[i] = (lab >= 0 && lab < K) ? (int32_t)new_index[lab] : -1;
    }
}

}  // namespace

size_t merge_ws_bytes(int64_t n, int64_t K) {
    const UpdDims u = upd_dims(n, K, 1, 1, 1);
    const int64_t nn = n > 0 ? n : 1;
    return align256((size_t)u.entries * 8) + align256((size_t)u.sblocks * 8) + align256((size_t)nn * 8) +
           align256((size_t)nn * 4) + align256((size_t)(K + 1) * 8);
}

hipError_t launch_merge_level(const LaunchCtx &c, const KSet &Z, int64_t n, const int32_t *labels,
                              const double *omega, int64_t n0, int32_t *C, int64_t *kept, int64_t *new_off,
                              void *new_points, void *new_weights, double *new_omega, void *ws) {
    const int64_t K = Z.n;
    const UpdDims u = upd_dims(n, K, 1, 1, 1);
    char *p = (char *)ws;
    int64_t *cnt = (int64_t *)p;
    p += align256((size_t)u.entries * 8);
    int64_t *bsum = (int64_t *)p;
    p += align256((size_t)u.sblocks * 8);
    int64_t *perm = (int64_t *)p;
    p += align256((size_t)(n > 0 ? n : 1) * 8);
    int32_t *skey = (int32_t *)p;
    p += align256((size_t)(n > 0 ? n : 1) * 4);
    int64_t *new_index = (int64_t *)p;
    const unsigned wave_blocks = (unsigned)((u.tiles + 3) / 4);
    const int64_t fill_grid = (u.entries + 255) / 256 < 4096 ? (u.entries + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_upd_fill, dim3((unsigned)fill_grid), dim3(256), 0, c.stream, cnt, u.entries);
    if (n > 0)
        hipLaunchKernelGGL(k_upd_count, dim3(wave_blocks), dim3(256), 0, c.stream, labels, n, K, u.tiles, cnt,
                           (int32_t *)nullptr);
    hipLaunchKernelGGL(k_upd_scan_blocks, dim3((unsigned)u.sblocks), dim3(256), 0, c.stream, cnt, u.entries, bsum);
    hipLaunchKernelGGL(k_upd_scan_top, dim3(1), dim3(1024), 0, c.stream, bsum, u.sblocks);
    hipLaunchKernelGGL(k_upd_scan_apply, dim3((unsigned)u.sblocks), dim3(256), 0, c.stream, cnt, u.entries, bsum);
    if (n > 0)
        hipLaunchKernelGGL(k_upd_place, dim3(wave_blocks), dim3(256), 0, c.stream, labels, n, K, u.tiles, cnt,
                           perm, skey);
    hipLaunchKernelGGL(k_merge_index, dim3(1), dim3(1024), 0, c.stream, cnt, K, u.tiles, Z.off, new_index, new_off,
                       kept);
    if (K > 0) {
        const int64_t g = (K + 255) / 256 < 4096 ? (K + 255) / 256 : 4096;
        hipLaunchKernelGGL(k_merge_weights, dim3((unsigned)g), dim3(256), 0, c.stream, cnt, perm, K, u.tiles, omega,
                           new_index, new_omega);
        const int64_t gw = (K + 3) / 4 < 65536 ? (K + 3) / 4 : 65536;
        if (Z.dtype == D2_F32)
            hipLaunchKernelGGL(k_merge_gather<float>, dim3((unsigned)gw), dim3(256), 0, c.stream, Z.off,
                               (const float *)Z.pts, (const float *)Z.w, Z.d, K, cnt, u.tiles, new_index, new_off,
                               (float *)new_points, (float *)new_weights);
        else
            hipLaunchKernelGGL(k_merge_gather<double>, dim3((unsigned)gw), dim3(256), 0, c.stream, Z.off,
                               (const double *)Z.pts, (const double *)Z.w, Z.d, K, cnt, u.tiles, new_index,
                               new_off, (double *)new_points, (double *)new_weights);
    }
    if (n0 > 0) {
        const int64_t g = (n0 + 255) / 256 < 4096 ? (n0 + 255) / 256 : 4096;
        hipLaunchKernelGGL(k_merge_inherit, dim3((unsigned)g), dim3(256), 0, c.stream, labels, n, K, new_index, C,
                           n0);
    }
    return hipGetLastError();
}

}  // namespace d2
