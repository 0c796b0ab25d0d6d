// Workgroup transportation simplex for supports beyond the lane-group
// shapes (65 .. 1024 atoms per side), used by d2_emd_batch, d2_assign and
// d2_pairwise when a set's declared max_support exceeds 64.  Same LP (Eq. (1), centroid fixed), same
// rules where they fix the result: weights divided by their index-order
// sums, direct-form FP64 costs, Bland's rule after 2(t+s) degenerate pivots
// in a row, a cap of max(50 t s, 100) pivots, stop when every reduced cost
// is >= -opt_tol * max C.  The entering cell is chosen by block pricing
// rather than over every cell (see below).
//
// One workgroup of 256 threads owns a pair at a time (persistent over the
// pair list).  The t x s cost matrix lives in the workgroup's slab of the
// caller's workspace; the basis tree lives in LDS as parent pointers over
// the t + s nodes (rows 0..t-1, columns t..t+s-1), each node holding the
// flow and the cost of the cell that joins it to its parent.  Per pivot:
//   * potentials and depths by pointer jumping over the parent pointers
//     (log2(t+s) rounds, every node in parallel): a node's potential is an
//     alternating sum of the costs on its root path;
//   * block pricing: cells in chunks of 2,048 from where the last search
//     stopped, the most negative reduced cost of the first chunk holding one
//     entering, so a pivot reads a chunk of the cost slab, not all of it;
//     optimality is a full cycle of chunks with none;
//   * wave 0 walks the tree path between the entering row and column (by
//     depth, all lanes in step), takes the ratio test on the edges at odd
//     distance from either end, moves the flow, and re-hangs the cut-off
//     part by reversing the parent pointers between the entering cell and
//     the leaving edge; the last three spread over its lanes.
// The start is the least-cost one (north-west corner under D2_INIT_NWC),
// built directly as a tree.  Every loop has a bound: pivots by the cap,
// tree walks by t + s steps, jumping by a fixed round count (a tree that
// does not resolve, or a tree walk that fails its checks, ends the pair
// with the internal-error status, kept apart from the pivot cap).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "d2_internal.h"

namespace d2 {

namespace {

constexpr int kWgMax = 1024;          // atoms per side, largest instance
constexpr int kWgSmall = 256;         // a smaller instance: 32 KB of LDS, four per CU
constexpr int kWgMid = 512;           // a middle one: 60 KB, two per CU
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kChunk = 2048;          // cells per pricing block
constexpr int kPer = kChunk / kThreads;   // cells of a block per thread
constexpr int kBatch = 8;             // of which loaded together
enum { kWOk = 0, kWBadWeights = 1, kWTooLarge = 2, kWPivotCap = 3, kWBadPoints = 4, kWInternal = 6 };

// LDS of one workgroup for supports up to CAP atoms per side.
template <int CAP>
struct WgMem {
    static constexpr int kNodes = 2 * CAP;
    int16_t par[kNodes];
    int16_t anc[2][kNodes];
    int16_t dep[2][kNodes];
    int8_t sg[2][kNodes];
    double off[2][kNodes];
    double pflow[kNodes];
    double ecost[kNodes];   // cost of the cell joining a node to its parent
    double pw[CAP], qw[CAP];
    int16_t pa[kNodes], pb[kNodes];
    double rv[kThreads];
    int32_t ri[kThreads];
    double cmax;
    int32_t bad, enter, stop, bland, status, scan;
    int32_t pend;   // a node still short of the root after the first jumping rounds
};

// One pointer-jumping round from bank `from` into the other bank: a node
// whose target is not the root adds its target's sum (with its own sign)
// and takes the target's target.  With `flag`, a node still short of the
// root after this round sets M.pend.
template <int CAP>
__device__ __forceinline__ void jump_round(WgMem<CAP> &M, int V, int tid, int from, bool flag) {
    const int to = 1 - from;
    for (int x = tid; x < V; x += kThreads) {
        const int an = M.anc[from][x];
        if (an >= 0) {
            M.off[to][x] = (double)M.sg[from][x] * M.off[from][an] + M.off[from][x];
            M.sg[to][x] = (int8_t)(M.sg[from][x] * M.sg[from][an]);
            M.anc[to][x] = M.anc[from][an];
            M.dep[to][x] = (int16_t)(M.dep[from][x] + M.dep[from][an]);
            if (flag && M.anc[from][an] >= 0) M.pend = 1;   // benign race: every writer stores 1
        } else {
            M.off[to][x] = M.off[from][x];
            M.sg[to][x] = M.sg[from][x];
            M.anc[to][x] = -1;
            M.dep[to][x] = M.dep[from][x];
        }
    }
}

template <typename T>
__device__ __forceinline__ double ldv(const void *p, int64_t i) {
    return (double)((const T *)p)[i];
}

// cost of the edge from node x to its parent
template <typename Mem>
__device__ __forceinline__ double edge_cost(const Mem &M, const double *C, int x, int T, int S) {
    const int y = M.par[x];
    return x < T ? C[(int64_t)x * S + (y - T)] : C[(int64_t)y * S + (x - T)];
}

// (v, c) beats the best so far (bv, bi): under Bland's rule the lower cell,
// else the lower reduced cost, then the lower cell; c = INT32_MAX is no
// candidate.
__device__ __forceinline__ bool better(double v, int c, double bv, int bi, bool bland) {
    if (c == INT32_MAX) return false;
    return bland ? c < bi : (v < bv || (v == bv && c < bi));
}

// Lane exchange within rows of 16 lanes (DPP): CTRL 0xB1 swaps neighbours,
// 0x4E swaps pairs, 0x141 mirrors each half row, 0x140 each row.
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)dpp_i32<CTRL>((int)(unsigned)u);
    const unsigned hi = (unsigned)dpp_i32<CTRL>((int)(unsigned)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int CTRL>
__device__ __forceinline__ void best_step(double &v, int &c, int &pay, bool bland) {
    const double ov = dpp_f64<CTRL>(v);
    const int oc = dpp_i32<CTRL>(c), op = dpp_i32<CTRL>(pay);
    if (better(ov, oc, v, c, bland)) { v = ov; c = oc; pay = op; }
}

// The best (v, c) of the 64 lanes of a wave under `better`, with a payload
// carried along, returned to every lane: four exchange steps leave each
// row of 16 with its best, then the four rows are compared.  Every lane of
// the wave must be active.
__device__ __forceinline__ void wave_best(double &v, int &c, int &pay, bool bland) {
    best_step<0xB1>(v, c, pay, bland);
    best_step<0x4E>(v, c, pay, bland);
    best_step<0x141>(v, c, pay, bland);
    best_step<0x140>(v, c, pay, bland);
    double bv = readlane_f64(v, 0);
    int bc = __builtin_amdgcn_readlane(c, 0), bp = __builtin_amdgcn_readlane(pay, 0);
    for (int r = 16; r < 64; r += 16) {
        const double ov = readlane_f64(v, r);
        const int oc = __builtin_amdgcn_readlane(c, r), op = __builtin_amdgcn_readlane(pay, r);
        if (better(ov, oc, bv, bc, bland)) { bv = ov; bc = oc; bp = op; }
    }
    v = bv; c = bc; pay = bp;
}

template <typename Mem>
__device__ __forceinline__ int edge_cell(const Mem &M, int x, int T, int S) {
    const int y = M.par[x];
    return x < T ? x * S + (y - T) : y * S + (x - T);
}

// Cheapest cell of row a over the open columns (lowest column on ties),
// by the 64 lanes of one wave; every lane returns the result.  `skip` is a
// column to leave out beyond the closed ones (-1 for none).
template <typename Mem>
__device__ __forceinline__ void row_min(const Mem &M, const double *C, int a, int T, int S, int skip, int lane,
                                        double &v, int &b) {
    v = INFINITY;
    b = INT32_MAX;
    for (int c = lane; c < S; c += 64)
        if (M.sg[0][T + c] && c != skip && better(C[(int64_t)a * S + c], c, v, b, false)) {
            v = C[(int64_t)a * S + c];
            b = c;
        }
    int unused = 0;
    wave_best(v, b, unused, false);
}

// Least-cost start (the cheapest cell over open rows and columns takes as
// much flow as its row and column have left; the line that runs out closes,
// the row on a tie unless it is the last open row or the last open column
// remains), built directly as a tree: each closed line hangs from the line
// its cell met, which closes later, so the t + s - 1 cells form a spanning
// tree rooted at the line that stays open.  Every row keeps its cheapest
// open cell; when a column closes, the rows whose cheapest cell was in it
// look again.  Scratch: off[0] the lines' remaining mass, off[1] and anc[1]
// the rows' cheapest cost and column, sg[0] the open flags.
template <typename Mem>
__device__ void lcm_start(Mem &M, const double *C, int T, int S, int tid) {
    const int V = T + S, lane = tid & 63, wave = tid >> 6;
    double *rest = M.off[0], *rmin = M.off[1];
    int16_t *rarg = M.anc[1];
    int8_t *open = M.sg[0];
    for (int x = tid; x < V; x += kThreads) {
        M.par[x] = -1;
        M.pflow[x] = 0.0;
        rest[x] = x < T ? M.pw[x] : M.qw[x - T];
        open[x] = 1;
    }
    __syncthreads();
    for (int a = wave; a < T; a += kWaves) {
        double v;
        int b;
        row_min(M, C, a, T, S, -1, lane, v, b);
        if (lane == 0) { rmin[a] = v; rarg[a] = (int16_t)b; }
    }
    __syncthreads();
    int nr = T, nc = S;
    int hold_i = -1, hold_j = 0;      // thread 0: the last step's remaining mass,
    double hold_ri = 0.0, hold_cj = 0.0;   // stored once every thread has read it
    for (int step = 0; step < V - 1; ++step) {
        if (tid == 0 && hold_i >= 0) { rest[hold_i] = hold_ri; rest[hold_j] = hold_cj; }
        // the cheapest open cell: lowest cost, then lowest cell index
        double best = INFINITY;
        int bc = INT32_MAX;
        for (int a = tid; a < T; a += kThreads)
            if (open[a] && better(rmin[a], a * S + rarg[a], best, bc, false)) { best = rmin[a]; bc = a * S + rarg[a]; }
        int unused = 0;
        wave_best(best, bc, unused, false);
        if (lane == 0) { M.rv[wave] = best; M.ri[wave] = bc; }
        __syncthreads();
        best = INFINITY;
        bc = INT32_MAX;
        for (int w = 0; w < kWaves; ++w)
            if (better(M.rv[w], M.ri[w], best, bc, false)) { best = M.rv[w]; bc = M.ri[w]; }
        if (bc == INT32_MAX) bc = 0;   // unreachable: an open row always has an open column
        const int i = bc / S, j = bc - (bc / S) * S;
        const double ri = rest[i], cj = rest[T + j], f = fmin(ri, cj);
        const bool close_row = (ri - f <= cj - f && nr > 1) || nc == 1;
        if (tid == 0) {
            hold_i = i; hold_ri = ri - f;
            hold_j = T + j; hold_cj = cj - f;
            const int closed = close_row ? i : T + j, other = close_row ? T + j : i;
            open[closed] = 0;
            M.par[closed] = (int16_t)other;
            M.pflow[closed] = f;
        }
        if (close_row) {
            --nr;
        } else {
            --nc;
            // rows whose cheapest cell was in column j look again
            for (int a0 = wave * 64; a0 < T; a0 += kThreads) {
                const int a = a0 + lane;
                uint64_t mask = __ballot(a < T && open[a] && rarg[a] == j);
                while (mask) {
                    const int r = a0 + __ffsll((unsigned long long)mask) - 1;
                    mask &= mask - 1;
                    double v;
                    int b;
                    row_min(M, C, r, T, S, j, lane, v, b);
                    if (lane == 0) { rmin[r] = v; rarg[r] = (int16_t)b; }
                }
            }
        }
        __syncthreads();
    }
}

// Pair k of the work: an explicit list, the cross product A x B (row-major,
// `ncols` = B.n), or the triangle i < j of one set (condensed row-major,
// `ncols` = n).
enum { kWgPairs = 0, kWgCross = 1, kWgTriangle = 2 };

__device__ __forceinline__ void wg_pair(int mode, const int64_t *pairs, int64_t ncols, int64_t k, int64_t &i,
                                        int64_t &j) {
    if (mode == kWgPairs) { i = pairs[2 * k]; j = pairs[2 * k + 1]; return; }
    if (mode == kWgCross) { i = k / ncols; j = k % ncols; return; }
    // row i holds n-1-i pairs; first guess from the closed form, then exact
    // integer steps (a handful at most)
    const int64_t n = ncols;
    double r = floor((2.0 * n - 1.0 - sqrt((2.0 * n - 1.0) * (2.0 * n - 1.0) - 8.0 * (double)k)) * 0.5);
    int64_t ii = (int64_t)r;
    if (ii < 0) ii = 0;
    if (ii > n - 2) ii = n - 2;
    for (int step = 0; step < 64 && ii > 0 && ii * n - ii * (ii + 1) / 2 > k; ++step) --ii;
    for (int step = 0; step < 64 && ii < n - 2 && (ii + 1) * n - (ii + 1) * (ii + 2) / 2 <= k; ++step) ++ii;
    i = ii;
    j = k - (ii * n - ii * (ii + 1) / 2) + ii + 1;
}

template <typename TIn, int CAP>
__global__ __launch_bounds__(kThreads) void k_emd_wg(KSet A, KSet B, int mode, const int64_t *pairs,
                                                      int64_t ncols, int64_t npairs, KOpts o, double *slabs,
                                                      int64_t slab_elems, double *dist,
                                                      const int64_t *plan_off, double *plan,
                                                      const int64_t *dual_off, double *duals, int32_t *status,
                                                      int32_t *pivots_out) {
    constexpr int kNodes = 2 * CAP;
    constexpr int kJumpRounds = CAP <= 256 ? 10 : CAP <= 512 ? 11 : 12;   // ceil(log2(2 CAP)) + 1
    // the first rounds resolve every node of depth < 2^kFirstRounds; the rest
    // run only when a node is still short of the root (same bank parity)
    constexpr int kFirstRounds = kJumpRounds - 4;
    __shared__ WgMem<CAP> M;
    const int tid = threadIdx.x;
    double *C = slabs + (int64_t)blockIdx.x * slab_elems;
    for (int64_t k = blockIdx.x; k < npairs; k += gridDim.x) {
        int64_t i, j;
        wg_pair(mode, pairs, ncols, k, i, j);
        int64_t t = -1, s = -1, a0 = 0, b0 = 0;
        if (i >= 0 && i < A.n && j >= 0 && j < B.n) {
            a0 = A.off[i]; b0 = B.off[j];
            t = A.off[i + 1] - a0; s = B.off[j + 1] - b0;
        }
        if (tid == 0 && pivots_out) { pivots_out[2 * k] = 0; pivots_out[2 * k + 1] = 0; }
        if (t < 1 || s < 1 || t > CAP || s > CAP || t * s > slab_elems) {   // uniform
            if (tid == 0) { dist[k] = __builtin_nan(""); if (status) status[k] = kWTooLarge; }
            continue;
        }
        const int T = (int)t, S = (int)s, V = T + S;
        // weights: validated, divided by their index-order sums
        for (int a = tid; a < T; a += kThreads) M.pw[a] = ldv<TIn>(A.w, a0 + a);
        for (int b = tid; b < S; b += kThreads) M.qw[b] = ldv<TIn>(B.w, b0 + b);
        if (tid == 0) { M.bad = 0; M.cmax = 0.0; M.status = kWOk; M.bland = 0; M.scan = 0; }
        __syncthreads();
        if (tid == 0) {
            double sp = 0.0, sq = 0.0;
            int bad = 0;
            for (int a = 0; a < T; ++a) { const double w = M.pw[a]; bad |= !(isfinite(w) && w >= 0.0); sp += w; }
            for (int b = 0; b < S; ++b) { const double w = M.qw[b]; bad |= !(isfinite(w) && w >= 0.0); sq += w; }
            bad |= !(sp > 0.0 && isfinite(sp) && sq > 0.0 && isfinite(sq));
            M.bad = bad;
            M.rv[0] = sp; M.rv[1] = sq;
        }
        __syncthreads();
        if (M.bad) {
            if (tid == 0) { dist[k] = __builtin_nan(""); if (status) status[k] = kWBadWeights; }
            __syncthreads();
            continue;
        }
        const double sp = M.rv[0], sq = M.rv[1];
        __syncthreads();
        for (int a = tid; a < T; a += kThreads) M.pw[a] = M.pw[a] / sp;
        for (int b = tid; b < S; b += kThreads) M.qw[b] = M.qw[b] / sq;
        // costs C_ab = sum_k (x_ak - y_bk)^2, k ascending
        const int d = A.d;
        double cm = 0.0;
        int nonfinite = 0;
        for (int c = tid; c < T * S; c += kThreads) {
            const int a = c / S, b = c % S;
            double acc = 0.0;
            for (int q = 0; q < d; ++q) {
                const double diff = ldv<TIn>(A.pts, (a0 + a) * d + q) - ldv<TIn>(B.pts, (b0 + b) * d + q);
                acc = fma(diff, diff, acc);
            }
            C[c] = acc;
            nonfinite |= !isfinite(acc);
            cm = fmax(cm, acc);
        }
        M.rv[tid] = cm;
        M.ri[tid] = nonfinite;
        __syncthreads();
        if (tid == 0) {
            double mx = 0.0;
            int nf = 0;
            for (int q = 0; q < kThreads; ++q) { mx = fmax(mx, M.rv[q]); nf |= M.ri[q]; }
            M.cmax = mx;
            M.bad = nf;
        }
        __syncthreads();
        if (tid == 0 && !M.bad && o.init == kStartNWC) {
            // north-west corner, built as a tree rooted at row 0
            for (int x = 0; x < V; ++x) { M.par[x] = -1; M.pflow[x] = 0.0; }
            int a = 0, b = 0, child = T;
            double rr = M.pw[0], rc = M.qw[0];
            M.par[T] = 0;
            for (int step = 0; step < V; ++step) {
                const double f = fmin(rr, rc);
                M.pflow[child] = f;
                rr -= f;
                rc -= f;
                if (a == T - 1 && b == S - 1) break;
                if ((rr <= rc && a < T - 1) || b == S - 1) {
                    ++a; rr = M.pw[a]; M.par[a] = (int16_t)(T + b); child = a;
                } else {
                    ++b; rc = M.qw[b]; M.par[T + b] = (int16_t)a; child = T + b;
                }
            }
        }
        __syncthreads();
        if (M.bad) {
            if (tid == 0) { dist[k] = __builtin_nan(""); if (status) status[k] = kWBadPoints; }
            __syncthreads();
            continue;
        }
        if (o.init != kStartNWC) lcm_start(M, C, T, S, tid);
        for (int x = tid; x < V; x += kThreads) M.ecost[x] = M.par[x] >= 0 ? edge_cost(M, C, x, T, S) : 0.0;
        const double delta = o.tol * M.cmax;
        int64_t cap = o.max_pivots > 0 ? o.max_pivots : 50LL * T * S;
        if (cap < 100) cap = 100;
        int64_t pivots = 0;
        int streak = 0, bland_pivots = 0;   // wave 0 only
        const int bland_after = o.bland_after > 0 ? o.bland_after : 2 * V;
        int buf = 0;
        for (;;) {
            // potentials and depths by pointer jumping
            for (int x = tid; x < V; x += kThreads) {
                const int y = M.par[x];
                M.anc[0][x] = (int16_t)y;
                M.sg[0][x] = y >= 0 ? -1 : 0;
                M.off[0][x] = y >= 0 ? M.ecost[x] : 0.0;
                M.dep[0][x] = y >= 0 ? 1 : 0;
            }
            if (tid == 0) M.pend = 0;
            __syncthreads();
#pragma unroll
            for (int rnd = 0; rnd < kFirstRounds; ++rnd) {
                jump_round(M, V, tid, rnd & 1, rnd == kFirstRounds - 1);
                __syncthreads();
            }
            if (M.pend) {
#pragma unroll
                for (int rnd = kFirstRounds; rnd < kJumpRounds; ++rnd) {
                    jump_round(M, V, tid, rnd & 1, false);
                    __syncthreads();
                }
            }
            buf = kJumpRounds & 1;   // extra rounds only copy resolved nodes
            // pricing by blocks: cells in chunks of kChunk, from where the
            // last search stopped and wrapping; the most negative reduced cost
            // of the first chunk holding one below -delta enters (lowest cell
            // on ties), and the pair is optimal once a full cycle of chunks
            // holds none.  Under Bland's rule one chunk covers every cell from
            // cell 0 and the lowest cell below -delta enters.  Basic cells
            // never enter: the jumping sums reach a tree edge's potentials in
            // another order than its cost, so its reduced cost is a rounding
            // residue rather than exactly 0, and a small tolerance could let
            // it through.  The chosen cell is checked once; a basic one joins
            // a short skip list (this pricing only) and the search runs again,
            // with the check inside the scan once the list is full.
            const bool bland = M.bland != 0;
            const int TS = T * S;
            int unresolved = 0;
            for (int x = tid; x < V; x += kThreads) unresolved |= M.anc[buf][x] >= 0;
            if (unresolved) M.bad = 1;   // benign race: every writer stores 1
            int pos = 0;
            const int width = bland ? TS : kChunk;
            double bv = -delta;
            int bi = INT32_MAX;
            int sk0 = -1, sk1 = -1, sk2 = -1, sk3 = -1;   // skipped basic cells (uniform)
            bool checked = false;
            for (;;) {
                pos = bland ? 0 : M.scan;
                bv = -delta;
                bi = INT32_MAX;
                for (int scanned = 0, rb = 0; scanned < TS; rb ^= 1) {   // >= 1 cell a pass
                    const int n = min(width, TS - scanned);
                    double best = -delta;
                    int bc = INT32_MAX;
                    if (!bland) {
                        // a chunk: at most kPer cells a thread, their loads issued
                        // together (a cell past the chunk reads cell 0, unused)
#pragma unroll
                        for (int e0 = 0; e0 < kPer; e0 += kBatch) {
                            double cv[kBatch];
                            int cc[kBatch];
#pragma unroll
                            for (int e = 0; e < kBatch; ++e) {
                                const int q = tid + (e0 + e) * kThreads;
                                int c = pos + q;
                                if (c >= TS) c -= TS;
                                cc[e] = q < n ? c : -1;
                                cv[e] = C[q < n ? c : 0];
                            }
#pragma unroll
                            for (int e = 0; e < kBatch; ++e) {
                                if (cc[e] >= 0) {
                                    const int c = cc[e], a = c / S, b = c - a * S;
                                    const double r = cv[e] - M.off[buf][a] - M.off[buf][T + b];
                                    if (r < -delta && better(r, c, best, bc, false) && c != sk0 && c != sk1 &&
                                        c != sk2 && c != sk3 &&
                                        (!checked || (M.par[a] != T + b && M.par[T + b] != a))) {
                                        best = r;
                                        bc = c;
                                    }
                                }
                            }
                        }
                    } else {
                        for (int q = tid; q < n; q += kThreads) {
                            const int a = q / S, b = q - a * S;   // one pass from cell 0
                            const double r = C[q] - M.off[buf][a] - M.off[buf][T + b];
                            if (r < -delta && better(r, q, best, bc, true) && q != sk0 && q != sk1 && q != sk2 &&
                                q != sk3 && (!checked || (M.par[a] != T + b && M.par[T + b] != a))) {
                                best = r;
                                bc = q;
                            }
                        }
                    }
                    int unused = 0;
                    wave_best(best, bc, unused, bland);
                    if ((tid & 63) == 0) {
                        M.rv[rb * kWaves + (tid >> 6)] = best;
                        M.ri[rb * kWaves + (tid >> 6)] = bc;
                    }
                    __syncthreads();   // two result banks: the next pass writes the other
                    for (int w = 0; w < kWaves; ++w)
                        if (better(M.rv[rb * kWaves + w], M.ri[rb * kWaves + w], bv, bi, bland)) {
                            bv = M.rv[rb * kWaves + w];
                            bi = M.ri[rb * kWaves + w];
                        }
                    scanned += n;
                    pos += n;
                    if (pos >= TS) pos -= TS;
                    if (bi != INT32_MAX) break;
                }
                if (bi == INT32_MAX || checked) break;
                const int ea = bi / S, eb = bi - ea * S;
                if (M.par[ea] != T + eb && M.par[T + eb] != ea) break;   // not a tree edge
                if (sk0 < 0) sk0 = bi;
                else if (sk1 < 0) sk1 = bi;
                else if (sk2 < 0) sk2 = bi;
                else if (sk3 < 0) sk3 = bi;
                else checked = true;
                __syncthreads();   // every thread has read the result banks before they are reused
            }
            if (tid < 64) {
                // wave 0 pivots: every lane takes the tree walk in step (one
                // lane stores the path); the ratio test, the flow update and
                // the re-hang spread over the lanes
                const int lane = tid;
                int stop = 0, stat = -1;
                if (M.bad) { stat = kWInternal; stop = 1; }
                else if (bi == INT32_MAX) stop = 1;
                else if (pivots >= cap) { stat = kWPivotCap; stop = 1; }
                else {
                    // tree path between row ei and column ej, by depth
                    const int ei = bi / S, ej = bi % S;
                    int x = ei, y = T + ej, na = 0, nb = 0;
                    const int16_t *dp = M.dep[buf];
                    bool ok = true;
                    // every step checks its node, so a damaged tree ends the
                    // pair instead of reading outside the arrays; the deeper
                    // end first climbs the depth difference (a parent is one
                    // shallower), then both climb until they meet
                    const int dx = dp[x], dy = dp[y];
                    for (int st = 0; st < V && ok && st < dx - dy; ++st) {
                        if (lane == 0) M.pa[na] = (int16_t)x;
                        ++na; x = M.par[x];
                        ok = x >= 0 && na < kNodes;
                    }
                    for (int st = 0; st < V && ok && st < dy - dx; ++st) {
                        if (lane == 0) M.pb[nb] = (int16_t)y;
                        ++nb; y = M.par[y];
                        ok = y >= 0 && nb < kNodes;
                    }
                    for (int st = 0; st < V && ok && x != y; ++st) {
                        if (lane == 0) { M.pa[na] = (int16_t)x; M.pb[nb] = (int16_t)y; }
                        ++na; x = M.par[x];
                        ++nb; y = M.par[y];
                        ok = x >= 0 && y >= 0 && na < kNodes && nb < kNodes;
                    }
                    if (!ok || x != y || na + nb < 3) { stat = kWInternal; stop = 1; }
                    else {
                        // ratio test over the edges at odd distance from either
                        // end: least flow, then lowest cell (unique)
                        double theta = INFINITY;
                        int lcell = INT32_MAX, lcode = 0;
                        for (int m = 2 * lane; m < na; m += 128) {
                            const int e = M.pa[m], ce = edge_cell(M, e, T, S);
                            if (better(M.pflow[e], ce, theta, lcell, false)) { theta = M.pflow[e]; lcell = ce; lcode = m; }
                        }
                        for (int m = 2 * lane; m < nb; m += 128) {
                            const int e = M.pb[m], ce = edge_cell(M, e, T, S);
                            if (better(M.pflow[e], ce, theta, lcell, false)) { theta = M.pflow[e]; lcell = ce; lcode = kNodes + m; }
                        }
                        wave_best(theta, lcell, lcode, false);
                        const int lside = lcode >= kNodes, lpos = lcode - lside * kNodes;
                        for (int m = lane; m < na; m += 64) M.pflow[M.pa[m]] += (m & 1) ? theta : -theta;
                        for (int m = lane; m < nb; m += 64) M.pflow[M.pb[m]] += (m & 1) ? theta : -theta;
                        // re-hang: reverse the parents from the entering end
                        // down to the leaving edge's child
                        const int16_t *path = lside == 0 ? M.pa : M.pb;
                        const int top = lside == 0 ? ei : T + ej;
                        const int other = lside == 0 ? T + ej : ei;
                        if (lpos < 64) {
                            // one step: the wave reads every old value before
                            // any lane writes
                            int xm = -1, xp = 0;
                            double fm = 0.0, em = 0.0;
                            if (lane >= 1 && lane <= lpos) {
                                xm = path[lane];
                                xp = path[lane - 1];
                                fm = M.pflow[xp];
                                em = M.ecost[xp];
                            }
                            if (xm >= 0) { M.pflow[xm] = fm; M.ecost[xm] = em; M.par[xm] = (int16_t)xp; }
                        } else if (lane == 0) {
                            for (int m = lpos; m >= 1; --m) {
                                M.pflow[path[m]] = M.pflow[path[m - 1]];
                                M.ecost[path[m]] = M.ecost[path[m - 1]];
                                M.par[path[m]] = path[m - 1];
                            }
                        }
                        if (lane == 0) {
                            M.pflow[top] = theta;
                            M.ecost[top] = C[(int64_t)ei * S + ej];
                            M.par[top] = (int16_t)other;
                        }
                        ++pivots;
                        bland_pivots += bland ? 1 : 0;
                        if (theta == 0.0) {
                            if (++streak >= bland_after && lane == 0) M.bland = 1;
                        } else {
                            streak = 0;
                            if (lane == 0) M.bland = 0;
                        }
                    }
                }
                if (lane == 0) {
                    M.stop = stop;
                    M.scan = pos;
                    if (stat >= 0) M.status = stat;
                }
            }
            __syncthreads();
            if (M.stop) break;
        }
        // objective over the basic cells, plan and duals
        if (tid == 0) {
            double obj = 0.0;
            if (M.status == kWOk)
                for (int x = 0; x < V; ++x)
                    if (M.par[x] >= 0) obj += M.pflow[x] * M.ecost[x];
            dist[k] = M.status == kWOk ? (o.want_sqrt ? sqrt(fmax(obj, 0.0)) : obj) : __builtin_nan("");
            if (status) status[k] = M.status;
            if (pivots_out) { pivots_out[2 * k] = (int32_t)pivots; pivots_out[2 * k + 1] = bland_pivots; }
        }
        if (M.status == kWOk) {
            if (plan) {
                double *P = plan + plan_off[k];
                for (int c = tid; c < T * S; c += kThreads) P[c] = 0.0;
                __syncthreads();
                for (int x = tid; x < V; x += kThreads)
                    if (M.par[x] >= 0) P[edge_cell(M, x, T, S)] = M.pflow[x];
            }
            if (duals) {
                double *D = duals + dual_off[k];
                for (int x = tid; x < V; x += kThreads) D[x] = M.off[buf][x];
            }
        }
        __syncthreads();
    }
}

}  // namespace

int wg_max_support() { return kWgMax; }

// Workgroups for a batch and the slab of each (t_max x s_max doubles),
// keeping the whole workspace within 1 GiB.  Supports up to kWgSmall run
// four workgroups per CU, up to kWgMid two, larger ones one.
void wg_plan(int64_t npairs, int tmax, int smax, int cu_count, int64_t *grid, int64_t *slab_elems) {
    const int64_t elems = (int64_t)(tmax > 0 ? tmax : 1) * (smax > 0 ? smax : 1);
    const int top = tmax > smax ? tmax : smax;
    const int per_cu = top <= kWgSmall ? 4 : top <= kWgMid ? 2 : 1;
    int64_t g = (int64_t)(cu_count > 0 ? cu_count : 256) * per_cu;
    const int64_t fit = (1LL << 30) / (elems * 8);
    if (g > fit) g = fit;
    if (g > npairs) g = npairs;
    if (g < 1) g = 1;
    *grid = g;
    *slab_elems = elems;
}

static hipError_t launch_wg(const LaunchCtx &c, const KSet &A, const KSet &B, int mode, const int64_t *pairs,
                            int64_t ncols, int64_t npairs, const KOpts &o, int tmax, int smax, double *dist,
                            const int64_t *plan_off, double *plan, const int64_t *dual_off, double *duals,
                            int32_t *status, int32_t *pivots, void *ws) {
    if (npairs == 0) return hipSuccess;
    int64_t grid, elems;
    wg_plan(npairs, tmax, smax, c.cu_count, &grid, &elems);
    const int top = tmax > smax ? tmax : smax;
#define D2_WG_LAUNCH(TIN, CAPV)                                                                                  \
    hipLaunchKernelGGL((k_emd_wg<TIN, CAPV>), dim3((unsigned)grid), dim3(kThreads), 0, c.stream, A, B, mode,    \
                       pairs, ncols, npairs, o, (double *)ws, elems, dist, plan_off, plan, dual_off, duals,        \
                       status, pivots)
    if (A.dtype == D2_F32) {
        if (top <= kWgSmall) D2_WG_LAUNCH(float, kWgSmall);
        else if (top <= kWgMid) D2_WG_LAUNCH(float, kWgMid);
        else D2_WG_LAUNCH(float, kWgMax);
    } else {
        if (top <= kWgSmall) D2_WG_LAUNCH(double, kWgSmall);
        else if (top <= kWgMid) D2_WG_LAUNCH(double, kWgMid);
        else D2_WG_LAUNCH(double, kWgMax);
    }
#undef D2_WG_LAUNCH
    return hipGetLastError();
}

hipError_t launch_emd_wg(const LaunchCtx &c, const KSet &A, const KSet &B, const int64_t *pairs, int64_t npairs,
                         const KOpts &o, int tmax, int smax, double *dist, const int64_t *plan_off, double *plan,
                         const int64_t *dual_off, double *duals, int32_t *status, int32_t *pivots, void *ws) {
    return launch_wg(c, A, B, kWgPairs, pairs, 0, npairs, o, tmax, smax, dist, plan_off, plan, dual_off, duals,
                     status, pivots, ws);
}

namespace {

// One wave per row of the n x K matrix: the minimum (lowest index on ties)
// and the worst status; label -1 when any pair of the row failed.
__global__ __launch_bounds__(256) void k_wg_argmin(const double *all, const int32_t *st, int64_t n, int64_t K,
                                                    int32_t *labels, double *best, int32_t *row_status) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; i < n; i += waves) {
        double v = INFINITY;
        int64_t jj = INT64_MAX;
        int worst = 0;
        for (int64_t j = lane; j < K; j += 64) {
            const double x = all[i * K + j];
            const int s = st[i * K + j];
            worst = s > worst ? s : worst;
            if (s == 0 && x < v) { v = x; jj = j; }
        }
        for (int sh = 32; sh >= 1; sh >>= 1) {
            const double ov = __shfl_xor(v, sh, 64);
            const int64_t oj = __shfl_xor(jj, sh, 64);
            const int ow = __shfl_xor(worst, sh, 64);
            if (ov < v || (ov == v && oj < jj)) { v = ov; jj = oj; }
            worst = ow > worst ? ow : worst;
        }
        if (lane == 0) {
            labels[i] = worst == 0 ? (int32_t)jj : -1;
            best[i] = worst == 0 ? v : __builtin_nan("");
            if (row_status) row_status[i] = worst;
        }
    }
}

}  // namespace

// Labelling with supports beyond the lane-group shapes: the cross product on
// the workgroup simplex into an n x K matrix, then the argmin per row.
// Workspace: slabs, then (unless `all` is given) the matrix, then statuses.
size_t wg_assign_bytes(int64_t n, int64_t K, int tmax, int smax, int cu_count) {
    int64_t grid, elems;
    wg_plan(n * K, tmax, smax, cu_count, &grid, &elems);
    const size_t slab = ((size_t)(grid * elems) * sizeof(double) + 255) & ~(size_t)255;
    const size_t mat = ((size_t)(n * K) * sizeof(double) + 255) & ~(size_t)255;
    return slab + mat + (size_t)(n * K) * sizeof(int32_t);
}

hipError_t launch_assign_wg(const LaunchCtx &c, const KSet &X, const KSet &Z, const KOpts &o, int tmax, int smax,
                            int32_t *labels, double *best, double *all, int32_t *row_status, void *ws) {
    const int64_t n = X.n, K = Z.n;
    if (n == 0) return hipSuccess;
    int64_t grid, elems;
    wg_plan(n * K, tmax, smax, c.cu_count, &grid, &elems);
    const size_t slab = ((size_t)(grid * elems) * sizeof(double) + 255) & ~(size_t)255;
    const size_t mat = ((size_t)(n * K) * sizeof(double) + 255) & ~(size_t)255;
    double *m = all ? all : (double *)((char *)ws + slab);
    int32_t *st = (int32_t *)((char *)ws + slab + mat);
    hipError_t e = launch_wg(c, X, Z, kWgCross, nullptr, K, n * K, o, tmax, smax, m, nullptr, nullptr, nullptr,
                             nullptr, st, nullptr, ws);
    if (e != hipSuccess) return e;
    const int64_t g = (n + 3) / 4 < 65536 ? (n + 3) / 4 : 65536;
    hipLaunchKernelGGL(k_wg_argmin, dim3((unsigned)g), dim3(256), 0, c.stream, m, st, n, K, labels, best,
                       row_status);
    return hipGetLastError();
}

// All pairs i < j of one set with supports beyond the lane-group shapes.
size_t wg_pairwise_bytes(int64_t n, int tmax, int cu_count) {
    int64_t grid, elems;
    wg_plan(n * (n - 1) / 2, tmax, tmax, cu_count, &grid, &elems);
    return (size_t)(grid * elems) * sizeof(double);
}

hipError_t launch_pairwise_wg(const LaunchCtx &c, const KSet &X, const KOpts &o, int tmax, double *condensed,
                              int32_t *status, void *ws) {
    const int64_t m = X.n * (X.n - 1) / 2;
    return launch_wg(c, X, X, kWgTriangle, nullptr, X.n, m, o, tmax, tmax, condensed, nullptr, nullptr, nullptr,
                     nullptr, status, nullptr, ws);
}

}  // namespace d2
