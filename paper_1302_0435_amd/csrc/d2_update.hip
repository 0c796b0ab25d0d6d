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
//   start    member 0 sends each atom to its cheapest centroid atom, which
//            fixes p_z (all s weights basic); every later member is the
//            north-west corner from its weights to p_z.  The basis matrix is
//            block triangular with non-singular blocks, so it is a basis;
//   pivots   explicit inverse of the basis: y = c_B B^-1, Dantzig's entering
//            column (Bland's after a run of degenerate pivots), the column
//            B^-1 a_q, the ratio test (least ratio, then lowest variable),
//            and the rank-one update of B^-1; B^-1 is rebuilt by Gauss-Jordan
//            elimination with partial pivoting every kRefactor pivots and
//            before optimality is declared; values of the solution at or
//            below kFlowEps are rounding noise of zeros and set to 0;
//   Step 2   each atom moves to the omega-and-flow-weighted mean of the
//            member atoms matched to it (Eq. (4)); Step 3 evaluates the
//            objective with the moved atoms and the same matchings.
// The dense arrays of a cluster (B, B^-1, costs, solution) live in the
// workgroup's slab of the workspace, sized for the caller's bound on the
// members of one cluster.  Every reduction runs in a fixed order.

namespace {

constexpr int kFreeThreads = 256;
constexpr int kRefactor = 64;
constexpr double kFreeTol = 1e-13;     // reduced costs above -kFreeTol max|c| count as >= 0
constexpr double kPivTol = 1e-9;       // least |entry| of B^-1 a_q taken in the ratio test
constexpr double kFlowEps = 1e-14;     // flows at or below this (of a unit mass) are zeros
enum { kFOk = 0, kFBadWeights = 1, kFTooLarge = 2, kFPivotCap = 3, kFInternal = 6 };

struct FreeDims {
    int nmax, xmax, zmax, d;
    int64_t mmax, vmax;
    size_t slab;
};

FreeDims free_dims(int nmax, int xmax, int zmax, int d) {
    FreeDims f;
    f.nmax = nmax > 0 ? nmax : 1;
    f.xmax = xmax > 0 ? xmax : 1;
    f.zmax = zmax > 0 ? zmax : 1;
    f.d = d;
    f.mmax = (int64_t)f.nmax * (f.xmax + f.zmax - 1) + 1;
    f.vmax = (int64_t)f.zmax * f.nmax * f.xmax + f.zmax;
    f.slab = 2 * align256((size_t)f.mmax * f.mmax * 8) + 2 * align256((size_t)f.vmax * 8) + align256((size_t)f.vmax) +
             5 * align256((size_t)f.mmax * 8) + align256((size_t)f.mmax * 4) + align256((size_t)(f.nmax + 1) * 4) +
             3 * align256((size_t)f.nmax * 8);
    return f;
}

struct FreeSlab {
    double *B, *Binv, *cost, *x, *xB, *y, *alpha, *b, *prow;
    int8_t *basic;
    int32_t *basis, *T;
    int64_t *obj;
    double *om, *isum;
};

__host__ __device__ inline FreeSlab free_slab(char *base, const FreeDims &f) {
    FreeSlab s;
    size_t off = 0;
    auto take = [&](size_t bytes) { char *q = base + off; off += (bytes + 255) & ~(size_t)255; return q; };
    s.B = (double *)take((size_t)f.mmax * f.mmax * 8);
    s.Binv = (double *)take((size_t)f.mmax * f.mmax * 8);
    s.cost = (double *)take((size_t)f.vmax * 8);
    s.x = (double *)take((size_t)f.vmax * 8);
    s.basic = (int8_t *)take((size_t)f.vmax);
    s.xB = (double *)take((size_t)f.mmax * 8);
    s.y = (double *)take((size_t)f.mmax * 8);
    s.alpha = (double *)take((size_t)f.mmax * 8);
    s.b = (double *)take((size_t)f.mmax * 8);
    s.prow = (double *)take((size_t)f.mmax * 8);
    s.basis = (int32_t *)take((size_t)f.mmax * 4);
    s.T = (int32_t *)take((size_t)(f.nmax + 1) * 4);
    s.obj = (int64_t *)take((size_t)f.nmax * 8);
    s.om = (double *)take((size_t)f.nmax * 8);
    s.isum = (double *)take((size_t)f.nmax * 8);
    return s;
}

struct FreeShared {
    double rv[kFreeThreads / 64];
    int ri[kFreeThreads / 64];
    int n, s, m, nvar, nw, stat, q, p, fresh, done, bland;
    double cmax, delta, theta;
};

// Block-wide (value, key) minimum, lowest key among equal values; keys of
// INT32_MAX are no candidates.  Every thread receives the result.
__device__ __forceinline__ void free_argmin(FreeShared &sh, double &v, int &k) {
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int ok = __shfl_xor(k, off, 64);
        if (ov < v || (ov == v && ok < k)) { v = ov; k = ok; }
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) { sh.rv[w] = v; sh.ri[w] = k; }
    __syncthreads();
    v = sh.rv[0];
    k = sh.ri[0];
    for (int q = 1; q < kFreeThreads / 64; ++q)
        if (sh.rv[q] < v || (sh.rv[q] == v && sh.ri[q] < k)) { v = sh.rv[q]; k = sh.ri[q]; }
}

__device__ __forceinline__ double free_max(FreeShared &sh, double v) {
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh.rv[w] = v;
    __syncthreads();
    double m = sh.rv[0];
    for (int q = 1; q < kFreeThreads / 64; ++q) m = fmax(m, sh.rv[q]);
    return m;
}

// Row of member k's coupling constraint for atom r, or -1 (dropped).
__device__ __forceinline__ int free_colrow(int sumt, int s, int k, int r) {
    if (k == 0) return sumt + r;
    if (r == s - 1) return -1;
    return sumt + s + (k - 1) * (s - 1) + r;
}

// Member of variable v < nw (binary search over the atom offsets T).
__device__ __forceinline__ int free_member(const int32_t *T, int n, int s, int v) {
    const int atom = v / s;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (T[mid] <= atom) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Rebuild B from the basis, B^-1 by Gauss-Jordan with partial pivoting, and
// x_B = B^-1 b.  Returns false when a pivot is (numerically) zero.
__device__ bool free_refactor(FreeShared &sh, const FreeSlab &S) {
    const int m = sh.m, n = sh.n, s = sh.s, nw = sh.nw, sumt = S.T[n];
    const int tid = threadIdx.x;
    for (int64_t e = tid; e < (int64_t)m * m; e += kFreeThreads) {
        S.B[e] = 0.0;
        S.Binv[e] = (e / m == e % m) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int j = tid; j < m; j += kFreeThreads) {   // column j of B: the basis variable's column
        const int v = S.basis[j];
        if (v < nw) {
            const int k = free_member(S.T, n, s, v);
            const int a = v / s - S.T[k], r = v % s;
            S.B[(int64_t)(S.T[k] + a) * m + j] = 1.0;
            const int cr = free_colrow(sumt, s, k, r);
            if (cr >= 0) S.B[(int64_t)cr * m + j] = 1.0;
        } else {
            const int r = v - nw;
            for (int k = 0; k < n; ++k) {
                const int cr = free_colrow(sumt, s, k, r);
                if (cr >= 0) S.B[(int64_t)cr * m + j] = -1.0;
            }
        }
    }
    __syncthreads();
    for (int c = 0; c < m; ++c) {
        double v = -1.0;
        int k = INT32_MAX;
        for (int i = c + tid; i < m; i += kFreeThreads) {
            const double a = fabs(S.B[(int64_t)i * m + c]);
            if (a > v || (a == v && i < k)) { v = a; k = i; }
        }
        // largest |entry| (lowest row on ties): argmin of the negation
        double nv = -v;
        free_argmin(sh, nv, k);
        if (!(-nv > 1e-12)) return false;
        const int pr = k;
        if (pr != c)
            for (int j = tid; j < m; j += kFreeThreads) {
                const double t1 = S.B[(int64_t)c * m + j];
                S.B[(int64_t)c * m + j] = S.B[(int64_t)pr * m + j];
                S.B[(int64_t)pr * m + j] = t1;
                const double t2 = S.Binv[(int64_t)c * m + j];
                S.Binv[(int64_t)c * m + j] = S.Binv[(int64_t)pr * m + j];
                S.Binv[(int64_t)pr * m + j] = t2;
            }
        __syncthreads();
        const double piv = S.B[(int64_t)c * m + c];
        __syncthreads();
        for (int j = tid; j < m; j += kFreeThreads) {
            S.B[(int64_t)c * m + j] /= piv;
            S.Binv[(int64_t)c * m + j] /= piv;
        }
        for (int i = tid; i < m; i += kFreeThreads) S.alpha[i] = S.B[(int64_t)i * m + c];   // factors, read first
        __syncthreads();
        for (int64_t e = tid; e < (int64_t)m * m; e += kFreeThreads) {
            const int i = (int)(e / m), j = (int)(e % m);
            if (i == c) continue;
            const double f = S.alpha[i];
            if (f != 0.0) {
                S.B[e] -= f * S.B[(int64_t)c * m + j];
                S.Binv[e] -= f * S.Binv[(int64_t)c * m + j];
            }
        }
        __syncthreads();
    }
    for (int i = tid; i < m; i += kFreeThreads) {
        double acc = 0.0;
        for (int j = 0; j < m; ++j) acc = fma(S.Binv[(int64_t)i * m + j], S.b[j], acc);
        S.xB[i] = acc < 0.0 ? 0.0 : acc;
    }
    __syncthreads();
    return true;
}

template <typename TIn>
__global__ __launch_bounds__(kFreeThreads) void k_free_solve(KSet X, KSet Z, KOpts o, const int64_t *pre,
                                                             const int64_t *perm, int64_t tiles, FreeDims f,
                                                             char *slabs, const double *objw, double *z_new,
                                                             double *w_new, double *eps1, double *eps3,
                                                             int32_t *counts, int32_t *obj_status,
                                                             int32_t *cluster_status) {
    __shared__ FreeShared sh;
    const int tid = threadIdx.x;
    const FreeSlab S = free_slab(slabs + (size_t)blockIdx.x * f.slab, f);
    const int d = X.d;
    for (int64_t j = blockIdx.x; j < Z.n; j += gridDim.x) {
        const int64_t pb = pre[j * tiles], pe = pre[(j + 1) * tiles];
        const int64_t z0 = Z.off[j];
        const int s = (int)(Z.off[j + 1] - z0);
        // centroid outputs default to the input (kept when the LP is not solved)
        for (int64_t e = tid; e < (int64_t)s * d; e += kFreeThreads)
            z_new[z0 * d + e] = ldw<TIn>(Z.pts, z0 * d + e);
        for (int r = tid; r < s; r += kFreeThreads) w_new[z0 + r] = ldw<TIn>(Z.w, z0 + r);
        // members: validate weights (thread per member), then compact in order
        const int64_t nall = pe - pb;
        if (tid == 0) { sh.stat = kFOk; sh.n = 0; }
        __syncthreads();
        if (nall > f.nmax || s < 1 || s > f.zmax) {
            for (int64_t q = pb + tid; q < pe; q += kFreeThreads)
                if (obj_status) obj_status[perm[q]] = kFTooLarge;
            if (tid == 0) {
                if (eps1) eps1[j] = __builtin_nan("");
                if (eps3) eps3[j] = __builtin_nan("");
                if (counts) counts[j] = 0;
                if (cluster_status) cluster_status[j] = kFTooLarge;
            }
            __syncthreads();
            continue;
        }
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
            S.isum[q - pb] = bad ? -1.0 : (om > 0.0 ? 1.0 / sum : 0.0);
            S.om[q - pb] = om;
        }
        __syncthreads();
        if (tid == 0) {
            int n = 0, acc = 0;
            for (int64_t q = 0; q < nall; ++q) {
                if (!(S.isum[q] > 0.0)) continue;   // invalid, or omega = 0: no part in the LP
                const int64_t i = perm[pb + q];
                S.obj[n] = i;
                S.om[n] = S.om[q];
                S.isum[n] = S.isum[q];
                S.T[n] = acc;
                acc += (int)(X.off[i + 1] - X.off[i]);
                ++n;
            }
            S.T[n] = acc;
            sh.n = n;
            sh.s = s;
            sh.m = acc + n * (s - 1) + 1;
            sh.nw = s * acc;
            sh.nvar = s * acc + s;
        }
        __syncthreads();
        const int n = sh.n, m = sh.m, nw = sh.nw, nvar = sh.nvar, sumt = S.T[n];
        if (n == 0) {
            if (tid == 0) {
                if (eps1) eps1[j] = 0.0;
                if (eps3) eps3[j] = 0.0;
                if (counts) counts[j] = 0;
                if (cluster_status) cluster_status[j] = kFOk;
            }
            __syncthreads();
            continue;
        }
        // costs omega_k |z_r - v_ka|^2 (direct form, coordinates ascending)
        double cm = 0.0;
        for (int v = tid; v < nvar; v += kFreeThreads) {
            double c = 0.0;
            if (v < nw) {
                const int k = free_member(S.T, n, s, v);
                const int a = v / s - S.T[k], r = v % s;
                const int64_t xa = (X.off[S.obj[k]] + a) * d, zr = (z0 + r) * d;
                double acc = 0.0;
                for (int qd = 0; qd < d; ++qd) {
                    const double diff = ldw<TIn>(X.pts, xa + qd) - ldw<TIn>(Z.pts, zr + qd);
                    acc = fma(diff, diff, acc);
                }
                c = S.om[k] * acc;
            }
            S.cost[v] = c;
            S.basic[v] = 0;
            cm = fmax(cm, fabs(c));
        }
        cm = free_max(sh, cm);
        if (tid == 0) { sh.cmax = cm; sh.delta = kFreeTol * cm; }
        for (int i = tid; i < m; i += kFreeThreads) {   // right-hand sides: member weights, then zeros
            double bv = 0.0;
            if (i < sumt) {
                const int k = free_member(S.T, n, 1, i);
                bv = ldw<TIn>(X.w, X.off[S.obj[k]] + (i - S.T[k])) * S.isum[k];
            }
            S.b[i] = bv;
        }
        __syncthreads();
        // the structured starting basis (serial: O(sum t + n s) steps)
        if (tid == 0) {
            int nb = 0;
            const int t0 = S.T[1] - S.T[0];
            for (int a = 0; a < t0; ++a) {   // member 0: cheapest atom, lowest on ties
                int rb = 0;
                for (int r = 1; r < s; ++r)
                    if (S.cost[a * s + r] < S.cost[a * s + rb]) rb = r;
                S.basis[nb++] = a * s + rb;
                S.prow[a] = rb;   // scratch: chosen atom
            }
            for (int r = 0; r < s; ++r) S.y[r] = 0.0;   // scratch: p_z
            for (int a = 0; a < t0; ++a) S.y[(int)S.prow[a]] += S.b[a];
            for (int r = 0; r < s; ++r) S.basis[nb++] = nw + r;
            for (int k = 1; k < n; ++k) {
                const int tk = S.T[k + 1] - S.T[k];
                int a = 0, r = 0;
                double ra = S.b[S.T[k]], rc = S.y[0];
                for (int step = 0; step < tk + s; ++step) {
                    S.basis[nb++] = s * (S.T[k] + a) + r;
                    const double fl = fmin(ra, rc);
                    ra -= fl;
                    rc -= fl;
                    if (a == tk - 1 && r == s - 1) break;
                    if ((ra <= rc && a < tk - 1) || r == s - 1) { ++a; ra = S.b[S.T[k] + a]; }
                    else { ++r; rc = S.y[r]; }
                }
            }
            sh.stat = nb == m ? kFOk : kFInternal;
            for (int q = 0; q < nb && q < m; ++q) S.basic[S.basis[q]] = 1;
        }
        __syncthreads();
        if (sh.stat == kFOk && !free_refactor(sh, S) && tid == 0) sh.stat = kFInternal;
        __syncthreads();
        // the simplex
        const int64_t cap = o.max_pivots > 0 ? o.max_pivots : (50LL * m > 100 ? 50LL * m : 100LL);
        const int bland_after = o.bland_after > 0 ? o.bland_after : 2 * m;
        int64_t pivots = 0;
        int streak = 0, since = 0;
        if (tid == 0) { sh.fresh = 1; sh.bland = 0; }
        __syncthreads();
        while (sh.stat == kFOk) {
            // y = c_B B^-1
            for (int i = tid; i < m; i += kFreeThreads) {
                double acc = 0.0;
                for (int jj = 0; jj < m; ++jj) acc = fma(S.cost[S.basis[jj]], S.Binv[(int64_t)jj * m + i], acc);
                S.y[i] = acc;
            }
            __syncthreads();
            // pricing: Dantzig (least reduced cost, lowest variable), or
            // Bland (lowest variable below -delta)
            const bool bl = sh.bland != 0;
            const double delta = sh.delta;
            double bv = INFINITY;
            int bq = INT32_MAX;
            for (int v = tid; v < nvar; v += kFreeThreads) {
                if (S.basic[v]) continue;
                double dv;
                if (v < nw) {
                    const int k = free_member(S.T, n, s, v);
                    const int a = v / s - S.T[k], r = v % s;
                    const int cr = free_colrow(sumt, s, k, r);
                    dv = S.cost[v] - S.y[S.T[k] + a] - (cr >= 0 ? S.y[cr] : 0.0);
                } else {
                    const int r = v - nw;
                    double acc = 0.0;
                    for (int k = 0; k < n; ++k) {
                        const int cr = free_colrow(sumt, s, k, r);
                        if (cr >= 0) acc += S.y[cr];
                    }
                    dv = acc;   // 0 - y . a with a = -1 on the coupling rows
                }
                if (!(dv < -delta)) continue;
                const double key = bl ? 0.0 : dv;
                if (key < bv || (key == bv && v < bq)) { bv = key; bq = v; }
            }
            free_argmin(sh, bv, bq);
            if (bq == INT32_MAX) {
                if (sh.fresh) break;   // optimal with freshly factored B^-1
                __syncthreads();
                if (!free_refactor(sh, S)) { if (tid == 0) sh.stat = kFInternal; __syncthreads(); break; }
                if (tid == 0) sh.fresh = 1;
                since = 0;
                __syncthreads();
                continue;
            }
            if (pivots >= cap) { if (tid == 0) sh.stat = kFPivotCap; __syncthreads(); break; }
            // alpha = B^-1 a_q
            const int q = bq;
            for (int i = tid; i < m; i += kFreeThreads) {
                double acc = 0.0;
                if (q < nw) {
                    const int k = free_member(S.T, n, s, q);
                    const int a = q / s - S.T[k], r = q % s;
                    const int cr = free_colrow(sumt, s, k, r);
                    acc = S.Binv[(int64_t)i * m + S.T[k] + a] + (cr >= 0 ? S.Binv[(int64_t)i * m + cr] : 0.0);
                } else {
                    const int r = q - nw;
                    for (int k = 0; k < n; ++k) {
                        const int cr = free_colrow(sumt, s, k, r);
                        if (cr >= 0) acc -= S.Binv[(int64_t)i * m + cr];
                    }
                }
                S.alpha[i] = acc;
            }
            __syncthreads();
            // ratio test: least x_B / alpha over alpha > kPivTol, then lowest variable
            double tv = INFINITY;
            int tk = INT32_MAX;
            for (int i = tid; i < m; i += kFreeThreads) {
                const double al = S.alpha[i];
                if (al > kPivTol) {
                    const double r = S.xB[i] / al;
                    const int key = S.basis[i];
                    if (r < tv || (r == tv && key < tk)) { tv = r; tk = key; }
                }
            }
            free_argmin(sh, tv, tk);
            if (tk == INT32_MAX) { if (tid == 0) sh.stat = kFInternal; __syncthreads(); break; }
            // the row holding variable tk
            if (tid == 0) {
                int pr = -1;
                for (int i = 0; i < m; ++i) if (S.basis[i] == tk) { pr = i; break; }
                sh.p = pr;
                sh.theta = tv > 0.0 ? tv : 0.0;
            }
            __syncthreads();
            const int pr = sh.p;
            if (pr < 0) { __syncthreads(); if (tid == 0) sh.stat = kFInternal; __syncthreads(); break; }
            const double theta = sh.theta, ap = S.alpha[pr];
            for (int jj = tid; jj < m; jj += kFreeThreads) S.prow[jj] = S.Binv[(int64_t)pr * m + jj] / ap;
            __syncthreads();
            for (int64_t e = tid; e < (int64_t)m * m; e += kFreeThreads) {
                const int i = (int)(e / m), jj = (int)(e % m);
                S.Binv[e] = i == pr ? S.prow[jj] : S.Binv[e] - S.alpha[i] * S.prow[jj];
            }
            for (int i = tid; i < m; i += kFreeThreads) {
                const double xv = i == pr ? theta : S.xB[i] - theta * S.alpha[i];
                S.xB[i] = xv < 0.0 ? 0.0 : xv;
            }
            __syncthreads();
            if (tid == 0) {
                S.basic[S.basis[pr]] = 0;
                S.basic[q] = 1;
                S.basis[pr] = q;
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
                if (!free_refactor(sh, S)) { if (tid == 0) sh.stat = kFInternal; __syncthreads(); break; }
                if (tid == 0) sh.fresh = 1;
                since = 0;
            }
            __syncthreads();
        }
        __syncthreads();
        const int st = sh.stat;
        if (st != kFOk) {
            for (int k = tid; k < n; k += kFreeThreads)
                if (obj_status) obj_status[S.obj[k]] = st;
            if (tid == 0) {
                if (eps1) eps1[j] = __builtin_nan("");
                if (eps3) eps3[j] = __builtin_nan("");
                if (counts) counts[j] = 0;
                if (cluster_status) cluster_status[j] = st;
            }
            __syncthreads();
            continue;
        }
        // the solution, densely
        for (int v = tid; v < nvar; v += kFreeThreads) S.x[v] = 0.0;
        __syncthreads();
        for (int i = tid; i < m; i += kFreeThreads) S.x[S.basis[i]] = S.xB[i] > kFlowEps ? S.xB[i] : 0.0;
        __syncthreads();
        for (int r = tid; r < s; r += kFreeThreads) w_new[z0 + r] = S.x[nw + r];
        // Step 1 value, in variable order
        if (tid == 0) {
            double v1 = 0.0;
            for (int v = 0; v < nw; ++v) v1 = fma(S.cost[v], S.x[v], v1);
            if (eps1) eps1[j] = v1;
            if (counts) counts[j] = n;
            if (cluster_status) cluster_status[j] = kFOk;
        }
        // Step 2: each atom to the omega-and-flow-weighted mean (Eq. (4)),
        // members and atoms in order; an atom with no mass stays
        for (int e = tid; e < s * d; e += kFreeThreads) {
            const int r = e / d, qd = e % d;
            double num = 0.0, den = 0.0;
            for (int k = 0; k < n; ++k) {
                const int tk2 = S.T[k + 1] - S.T[k];
                const int64_t xa = X.off[S.obj[k]];
                double nk = 0.0, dk = 0.0;
                for (int a = 0; a < tk2; ++a) {
                    const double wv = S.x[s * (S.T[k] + a) + r];
                    nk = fma(wv, ldw<TIn>(X.pts, (xa + a) * d + qd), nk);
                    dk += wv;
                }
                num = fma(S.om[k], nk, num);
                den = fma(S.om[k], dk, den);
            }
            if (den > 0.0) z_new[(z0 + r) * d + qd] = num / den;
        }
        __syncthreads();
        // Step 3: the objective with the moved atoms and the same matchings
        if (tid == 0) {
            double v3 = 0.0;
            for (int v = 0; v < nw; ++v) {
                const double wv = S.x[v];
                if (wv == 0.0) continue;
                const int k = free_member(S.T, n, s, v);
                const int a = v / s - S.T[k], r = v % s;
                const int64_t xa = (X.off[S.obj[k]] + a) * d;
                double acc = 0.0;
                for (int qd = 0; qd < d; ++qd) {
                    const double diff = ldw<TIn>(X.pts, xa + qd) - z_new[(z0 + r) * d + qd];
                    acc = fma(diff, diff, acc);
                }
                v3 = fma(S.om[k] * wv, acc, v3);
            }
            if (eps3) eps3[j] = v3;
        }
        __syncthreads();
    }
}

}  // namespace

size_t update_free_slab_bytes(int max_members, int xmax, int zmax, int d) {
    return free_dims(max_members, xmax, zmax, d).slab;
}

size_t update_free_ws_bytes(int64_t n, int64_t K, int d, int xmax, int zmax, int max_members, int cu_count,
                            int64_t *grid_out) {
    const UpdDims u = upd_dims(n, K, d, xmax, zmax);
    const FreeDims f = free_dims(max_members, xmax, zmax, d);
    int64_t grid = (int64_t)(cu_count > 0 ? cu_count : 256) * 2;
    const int64_t fit = (int64_t)((size_t)1 << 30) / (int64_t)f.slab;
    if (grid > fit) grid = fit;
    if (grid > K) grid = K;
    if (grid < 1) grid = 1;
    if (grid_out) *grid_out = grid;
    // grouping arrays (counts, block sums, order) then the slabs
    return align256((size_t)u.entries * 8) + align256((size_t)u.sblocks * 8) + align256((size_t)(n > 0 ? n : 1) * 8) +
           align256((size_t)(n > 0 ? n : 1) * 4) + (size_t)grid * f.slab;
}

hipError_t launch_update_free(const LaunchCtx &c, const KSet &X, const KSet &Z, int xmax, int zmax,
                              int max_members, const KOpts &o, const int32_t *labels, const double *obj_weights,
                              double *z_new, double *w_new, double *eps1, double *eps3, int32_t *counts,
                              int32_t *obj_status, int32_t *cluster_status, void *ws) {
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
    char *slabs = p;
    const unsigned wave_blocks = (unsigned)((u.tiles + 3) / 4);
    const int64_t fill_grid = (u.entries + 255) / 256 < 4096 ? (u.entries + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_upd_fill, dim3((unsigned)fill_grid), dim3(256), 0, c.stream, cnt, u.entries);
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
    if (X.dtype == D2_F32)
        hipLaunchKernelGGL(k_free_solve<float>, dim3((unsigned)grid), dim3(kFreeThreads), 0, c.stream, X, Z, o, cnt,
                           perm, u.tiles, f, slabs, obj_weights, z_new, w_new, eps1, eps3, counts, obj_status,
                           cluster_status);
    else
        hipLaunchKernelGGL(k_free_solve<double>, dim3((unsigned)grid), dim3(kFreeThreads), 0, c.stream, X, Z, o, cnt,
                           perm, u.tiles, f, slabs, obj_weights, z_new, w_new, eps1, eps3, counts, obj_status,
                           cluster_status);
    return hipGetLastError();
}

}  // namespace d2
