// Wave-parallel transportation simplex for the squared Mallows distance.
//
// One pair (P, Q) is the LP of Eq. (1) with the centroid fixed (paper,
// Sec. 1.1): minimise sum_ab w_ab |x_a - y_b|^2 over w >= 0 with row sums p
// and column sums q.  The paper leaves the LP solver open; this file solves
// it with the transportation simplex (u-v method): a starting basis (least
// cost, north-west corner or Vogel), dual potentials u, v with u_a + v_b =
// C_ab on the basis, pricing r_ab = C_ab - u_a - v_b, and pivots around the
// cycle that the entering cell closes in the basis spanning tree.
//
// GPU mapping.  A "group" of G lanes (G = 16, 32 or 64; 64/G pairs per
// wavefront) owns one pair at a time.  The pair is oriented so that rows are
// the larger support (D^2 is symmetric); the column count is at most GS.
// Lane l owns row node l and column node l of the basis tree, and row l of
// the cost tile (in registers, or in an LDS tile for the widest shape).
// Each node stores its parent, the flow and cost of its parent edge, its
// potential and its ancestor set as a bitmask.  With ancestor masks a pivot
// needs no pointer chasing:
//   * the cycle of entering cell (r, c) is the tree path r..c, i.e. the nodes
//     in anc(r) xor anc(c); the edges whose flow decreases are the row nodes
//     on r's side and the column nodes on c's side;
//   * the ratio test is a group min-reduction over those edges' flows;
//   * the subtree cut off by the leaving edge is {x : L in anc(x)}, one
//     ballot; it is re-hung below the entering cell, the edges on the path
//     from the entering end up to L ("stem") change direction, and the new
//     ancestor set of every moved node is anc(p) | (A xor stem) | {y}, with A
//     its old ancestor set inside the subtree and y its deepest ancestor on
//     the stem (looked up by position along the stem);
//   * potentials change only inside the moved subtree, by +-r_entering.
// Potentials are set from the tree by pointer jumping at the start and once
// more before optimality is declared, so rounding drift in the incremental
// updates cannot end the solve early.
//
// Group communication: reductions are butterflies over DPP row permutations
// (16 lanes), plus a swizzle (32) and a lane permute (64); broadcasts go
// through a few LDS words, and the column points of the cost rows through an
// LDS staging area.  All loops are bounded: the start by the number of lines,
// the pivots by a cap that reports failure.
//
// Every arithmetic step that decides the result runs in an order that does
// not depend on the shape (index-order sums, exact min/max reductions), so
// all shapes return the same bits for the same pair.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "d2_internal.h"

namespace d2 {

enum { kOk = 0, kBadWeights = 1, kTooLarge = 2, kPivotCap = 3, kBadPoints = 4, kInternal = 6 };
constexpr int kNoKey = 0x7fffffff;

// ------------------------------------------------------------------ masks

// Node sets of one group's tree: rows are nodes 0..G-1, columns G..2G-1.
template <int G>
struct Mask;

template <>
struct Mask<16> {  // rows in bits [0,16), columns in [16,32)
    uint32_t m;
    __device__ static Mask none() { return {0u}; }
    __device__ static Mask node(int id) { return {1u << id}; }
    __device__ static Mask rows_only() { return {0x0000FFFFu}; }
    __device__ static Mask cols_only() { return {0xFFFF0000u}; }
    __device__ static Mask from_bits(uint64_t r, uint64_t c) { return {(uint32_t)r | ((uint32_t)c << 16)}; }
    __device__ Mask operator|(Mask o) const { return {m | o.m}; }
    __device__ Mask operator&(Mask o) const { return {m & o.m}; }
    __device__ Mask operator^(Mask o) const { return {m ^ o.m}; }
    __device__ Mask andnot(Mask o) const { return {m & ~o.m}; }
    __device__ bool has(int id) const { return (m >> id) & 1u; }
    __device__ int popc() const { return __popc(m); }
};

template <>
struct Mask<32> {  // rows in bits [0,32), columns in [32,64)
    uint64_t m;
    __device__ static Mask none() { return {0ull}; }
    __device__ static Mask node(int id) { return {1ull << id}; }
    __device__ static Mask rows_only() { return {0x00000000FFFFFFFFull}; }
    __device__ static Mask cols_only() { return {0xFFFFFFFF00000000ull}; }
    __device__ static Mask from_bits(uint64_t r, uint64_t c) { return {r | (c << 32)}; }
    __device__ Mask operator|(Mask o) const { return {m | o.m}; }
    __device__ Mask operator&(Mask o) const { return {m & o.m}; }
    __device__ Mask operator^(Mask o) const { return {m ^ o.m}; }
    __device__ Mask andnot(Mask o) const { return {m & ~o.m}; }
    __device__ bool has(int id) const { return (m >> id) & 1ull; }
    __device__ int popc() const { return __popcll(m); }
};

template <>
struct Mask<64> {  // one word for rows, one for columns
    uint64_t r, c;
    __device__ static Mask none() { return {0ull, 0ull}; }
    __device__ static Mask node(int id) { return id < 64 ? Mask{1ull << id, 0ull} : Mask{0ull, 1ull << (id - 64)}; }
    __device__ static Mask rows_only() { return {~0ull, 0ull}; }
    __device__ static Mask cols_only() { return {0ull, ~0ull}; }
    __device__ static Mask from_bits(uint64_t rr, uint64_t cc) { return {rr, cc}; }
    __device__ Mask operator|(Mask o) const { return {r | o.r, c | o.c}; }
    __device__ Mask operator&(Mask o) const { return {r & o.r, c & o.c}; }
    __device__ Mask operator^(Mask o) const { return {r ^ o.r, c ^ o.c}; }
    __device__ Mask andnot(Mask o) const { return {r & ~o.r, c & ~o.c}; }
    __device__ bool has(int id) const { return id < 64 ? ((r >> id) & 1ull) : ((c >> (id - 64)) & 1ull); }
    __device__ int popc() const { return __popcll(r) + __popcll(c); }
};

// Orders LDS traffic between lanes of one wavefront (the hardware executes a
// wavefront's LDS operations in order; this keeps the compiler from moving
// loads above stores).
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------- lane exchanges

// Butterfly partner exchange, step k of an all-reduce over G lanes:
// quad xor 1, quad xor 2, half-row mirror, row mirror (DPP), then xor 16
// (swizzle, G >= 32) and xor 32 (lane permute, G = 64).  After log2(G)
// steps with a commutative, associative combine every lane holds the result.
template <int STEP>
__device__ __forceinline__ int xchg(int v) {
    if constexpr (STEP == 0) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);
    else if constexpr (STEP == 1) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);
    else if constexpr (STEP == 2) return __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true);
    else if constexpr (STEP == 3) return __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true);
    else if constexpr (STEP == 4) return __builtin_amdgcn_ds_swizzle(v, 0x401F);
    else return __shfl_xor(v, 32, 64);
}

template <int STEP>
__device__ __forceinline__ double xchg(double v) {
    long long b = __double_as_longlong(v);
    int lo = xchg<STEP>((int)(b & 0xffffffffll));
    int hi = xchg<STEP>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int G>
struct Steps { static constexpr int n = G == 16 ? 4 : (G == 32 ? 5 : 6); };

template <int G, int STEP = 0>
__device__ __forceinline__ double group_min(double v) {
    if constexpr (STEP < Steps<G>::n) return group_min<G, STEP + 1>(fmin(v, xchg<STEP>(v)));
    else return v;
}

template <int G, int STEP = 0>
__device__ __forceinline__ int group_min_int(int v) {
    if constexpr (STEP < Steps<G>::n) return group_min_int<G, STEP + 1>(min(v, xchg<STEP>(v)));
    else return v;
}

template <int G, int STEP = 0>
__device__ __forceinline__ double group_max(double v) {
    if constexpr (STEP < Steps<G>::n) return group_max<G, STEP + 1>(fmax(v, xchg<STEP>(v)));
    else return v;
}

// (value, key) minimum over the group, lowest key on equal values: the
// exact minimum value first, then the least key among the lanes holding it.
template <int G>
__device__ __forceinline__ void group_argmin(double &v, int &k) {
    const double m = group_min<G>(v);
    k = group_min_int<G>(v == m ? k : kNoKey);
    v = m;
}

template <int J, int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (J < N) {
        f(std::integral_constant<int, J>{});
        static_for<J + 1, N>(f);
    }
}

// Maximum of a group-uniform value over the groups of the wavefront that are
// executing, as a scalar, so loops bounded by it branch on the scalar unit.
// A group whose loop has ended is inactive and its registers hold stale
// values, so only groups present in the active mask count (groups are
// always active or inactive as a whole).
template <int G>
__device__ __forceinline__ int wave_max(int v) {
    const uint64_t act = __ballot(1);
    int m = 0;
    static_for<0, 64 / G>([&](auto k) {
        constexpr int b = decltype(k)::value * G;
        const int x = __builtin_amdgcn_readlane(v, b);
        m = ((act >> b) & 1ull) ? max(m, x) : m;
    });
    return m;
}

template <int G>
__device__ __forceinline__ uint64_t group_bits(bool p, int gbase) {
    uint64_t b = __ballot(p);
    const uint64_t gm = G == 64 ? ~0ull : ((1ull << G) - 1ull);
    return (b >> gbase) & gm;
}


// f(integral_constant<int, N>) for the least N in {Q, 2Q, .., MAX} with
// N >= n.  With a wave-uniform n the choice is a few scalar branches and the
// body runs fully unrolled over N items, so loops over a pair's columns stop
// near its support instead of running to the shape's capacity (a plain
// guard inside an unrolled loop is turned into predicated selects).
template <int MAX, int Q, int N = Q, typename F>
__device__ __forceinline__ void up_to(int n, F &&f) {
    if constexpr (N >= MAX) {
        f(std::integral_constant<int, MAX>{});
    } else {
        if (n <= N) f(std::integral_constant<int, N>{});
        else up_to<MAX, Q, N + Q>(n, f);
    }
}

// ------------------------------------------------------------ group memory

// Coordinates per LDS staging round of the cost rows: 8 for the 32-lane
// shape, 4 for the others, whose register budgets are tighter (measured).
template <int G>
constexpr int stage_k() { return G == 32 ? 8 : 4; }

// The widest shape keeps columns [0, kSplitCols) of its cost row in
// registers and the rest in an LDS tile (TileHalf below).
constexpr int kSplitCols = 32;

template <int G, int GS>
struct GroupMem {
    alignas(16) double vpot[GS];  // column potentials, read by every row lane when pricing
    Mask<G> ancRm[G];        // ancestor masks of row nodes (mirror for broadcast)
    Mask<G> ancCm[GS];       // ancestor masks of column nodes
    double bc_r, bc_c;       // entering cell: reduced cost and cost
    long long grab;          // work-queue slot broadcast
    union {
        struct { double pw[G]; double qw[GS]; double P[G]; double Q[GS]; double colcpar[GS];
                 int colpar[GS]; int kind[2 * G]; int lastpos[2 * G]; } init;
        struct { int jmp[2 * G]; Mask<G> anc[2 * G]; double off[2 * G]; } jump;
        struct { int newpar[2 * G]; int stemtab[2 * G]; double newflow[2 * G];
                 double newcpar[2 * G]; } piv;
        struct { double obj[2 * G]; double colflow[GS]; int colpar[GS]; } fin;
        struct { alignas(16) double y[GS][stage_k<G>()]; } stage;   // column points, KC coordinates
        struct { unsigned long long key[GS]; int row[GS]; int shut[GS]; double x[GS]; double cost[GS];
                 double remR[G]; double remC[GS]; double lastrow[GS]; unsigned long long gkey; } lcm;
    } u;
};

// Cost tile, column-major C[b][a], for Vogel's start (which scans columns).
template <int G, int GS>
struct Tile { double C[GS][G + 1]; };
struct NoTile { char pad; };

// The widest shape's LDS tile of columns [kSplitCols, GS) (column-major,
// C[b - kSplitCols][a]), which halves the LDS a pair needs and lets two
// wavefronts share a SIMD.
template <int G, int GS>
struct TileHalf { double C[GS - kSplitCols][G]; };
template <typename T> struct IsTileHalf : std::false_type {};
template <int G, int GS> struct IsTileHalf<TileHalf<G, GS>> : std::true_type {};

// Per-lane state: row node l, column node l, and row l of the cost tile.
template <int G, int GS, bool LT>
struct NodeState {
    int parR, parC;          // parent index (a column / a row), -1 at the root
    double flowR, flowC;     // flow on the edge to the parent
    double cparR, cparC;     // cost of the edge to the parent
    double potR, potC;       // u_l, v_l
    Mask<G> ancR, ancC;      // ancestors including the node itself
    typename std::conditional<GS == 64, uint64_t, uint32_t>::type bas;  // basic cells of row l
    double crow[LT ? kSplitCols : GS];  // C[l][j] (LDS-tile shape: j < kSplitCols); +inf beyond
                                        // the columns and on rows beyond the support
};

template <typename T>
__device__ __forceinline__ double ldw(const void *p, int64_t i) {
    return (double)((const T *)p)[i];
}

// One oriented pair: rows = the larger support.
struct PairView {
    const void *xr, *wr;  // row side points/weights, already offset to the object
    const void *xc, *wc;  // column side
    int T, S;             // row / column support sizes
    bool swapped;         // rows are the second object (B side) of the pair
};

__device__ __forceinline__ PairView orient(const KSet &A, int64_t i, const KSet &B, int64_t j,
                                           int esize) {
    int64_t a0 = A.off[i], a1 = A.off[i + 1], b0 = B.off[j], b1 = B.off[j + 1];
    int64_t t = a1 - a0, s = b1 - b0;
    PairView v;
    const char *pa = (const char *)A.pts + a0 * A.d * esize;
    const char *pb = (const char *)B.pts + b0 * B.d * esize;
    const char *wa = (const char *)A.w + a0 * esize;
    const char *wb = (const char *)B.w + b0 * esize;
    long long tt = t < 0 ? -1 : (t > 1000000 ? 1000000 : t);
    long long ss = s < 0 ? -1 : (s > 1000000 ? 1000000 : s);
    if (tt >= ss) {
        v.xr = pa; v.wr = wa; v.T = (int)tt; v.xc = pb; v.wc = wb; v.S = (int)ss; v.swapped = false;
    } else {
        v.xr = pb; v.wr = wb; v.T = (int)ss; v.xc = pa; v.wc = wa; v.S = (int)tt; v.swapped = true;
    }
    return v;
}

// Cost of cell (l, j) from the lane's registers or the LDS tile; j must be
// a compile-time index wherever it can select a register.
template <int G, int GS, bool LT, typename TileT>
__device__ __forceinline__ double cost_at(const NodeState<G, GS, LT> &N, const TileT &tile, int l, int j) {
    if constexpr (LT && IsTileHalf<TileT>::value)
        return j < kSplitCols ? N.crow[j < kSplitCols ? j : 0] : tile.C[j - kSplitCols][l];
    else if constexpr (LT) return tile.C[j][l];
    else return N.crow[j];
}

template <int G, int GS, bool LT, typename TileT>
__device__ __forceinline__ void put_cost(NodeState<G, GS, LT> &N, TileT &tile, int l, int j, double c) {
    if constexpr (LT && IsTileHalf<TileT>::value) {
        if (j < kSplitCols) N.crow[j < kSplitCols ? j : 0] = c;
        else tile.C[j - kSplitCols][l] = c;
    } else if constexpr (LT) {
        tile.C[j][l] = c;
    } else {
        N.crow[j] = c;
    }
}

// Cost of cell (l, j) for a run-time j.
template <int G, int GS, bool LT, typename TileT>
__device__ __forceinline__ double cost_pick(const NodeState<G, GS, LT> &N, const TileT &tile, int l, int j) {
    if constexpr (LT && !IsTileHalf<TileT>::value) {
        return tile.C[j][l];
    } else {
        constexpr int RC = LT ? kSplitCols : GS;
        if constexpr (LT) {
            if (j >= RC) return tile.C[j - RC][l];
        }
        double r = 0.0;
#pragma unroll
        for (int k = 0; k < RC; ++k) r = (k == j) ? N.crow[k] : r;
        return r;
    }
}

// ------------------------------------------------------------ potentials

// Potentials (and, with MASKS, ancestor masks) from the parent pointers by
// pointer jumping.  A tree edge joins node x to its parent with the cost
// cpar(x) of their cell, and u_a + v_b = C_ab there gives
// pot(x) = cpar(x) - pot(parent(x)), with pot(root) = 0.  Every node keeps a
// target t(x) (first its parent), the parity of the path from x up to t(x)
// and an offset o(x) such that pot(x) = o(x) + (-1)^parity pot(t(x)).  A
// round replaces t(x) by t(t(x)) and folds o(t(x)) into o(x); after
// ceil(log2 2G) rounds every target is the root and pot(x) = o(x).  The order
// of the additions follows the tree alone, so every group width computes the
// same bits.  Also refreshes the LDS mirrors read when pricing and when
// broadcasting the entering cell.
template <int G, int GS, bool LT, bool MASKS>
__device__ __forceinline__ void tree_jump(GroupMem<G, GS> &M, NodeState<G, GS, LT> &N, int l, int T, int S) {
    const bool hasR = l < T, hasC = l < S;
    const int idR = l, idC = G + l;
    const bool pR = hasR && N.parR >= 0, pC = hasC && N.parC >= 0;
    constexpr int kOdd = 1 << 30;   // parity bit beside the target index
    int jR = pR ? (G + N.parR) | kOdd : idR;
    int jC = pC ? N.parC | kOdd : idC;
    double oR = pR ? N.cparR : 0.0, oC = pC ? N.cparC : 0.0;
    Mask<G> aR = hasR ? Mask<G>::node(idR) : Mask<G>::none();
    Mask<G> aC = hasC ? Mask<G>::node(idC) : Mask<G>::none();
    M.u.jump.jmp[idR] = jR;
    M.u.jump.jmp[idC] = jC;
    M.u.jump.off[idR] = oR;
    M.u.jump.off[idC] = oC;
    if constexpr (MASKS) {
        M.u.jump.anc[idR] = aR;
        M.u.jump.anc[idC] = aC;
    }
    wsync();
#pragma unroll 1
    for (int k = 0; k < Steps<G>::n + 1; ++k) {
        const int tR = jR & (kOdd - 1), tC = jC & (kOdd - 1);
        const int nR = M.u.jump.jmp[tR], nC = M.u.jump.jmp[tC];
        const double xR = M.u.jump.off[tR], xC = M.u.jump.off[tC];
        Mask<G> mR, mC;
        if constexpr (MASKS) {
            mR = M.u.jump.anc[tR];
            mC = M.u.jump.anc[tC];
        }
        wsync();
        oR = (jR & kOdd) ? oR - xR : oR + xR;
        oC = (jC & kOdd) ? oC - xC : oC + xC;
        jR = nR ^ (jR & kOdd);
        jC = nC ^ (jC & kOdd);
        M.u.jump.jmp[idR] = jR;
        M.u.jump.jmp[idC] = jC;
        M.u.jump.off[idR] = oR;
        M.u.jump.off[idC] = oC;
        if constexpr (MASKS) {
            aR = aR | mR;
            aC = aC | mC;
            M.u.jump.anc[idR] = aR;
            M.u.jump.anc[idC] = aC;
        }
        wsync();
    }
    N.potR = hasR ? oR : 0.0;
    N.potC = hasC ? oC : 0.0;
    if constexpr (MASKS) {
        N.ancR = aR;
        N.ancC = aC;
    }
    M.ancRm[l] = N.ancR;
    if (l < GS) {
        if (hasC) M.vpot[l] = N.potC;
        M.ancCm[l] = N.ancC;
    }
    wsync();
}

// ------------------------------------------------------------ one solve

// Integer key with the order of the double: negative values have every bit
// flipped, others only the sign bit.
__device__ __forceinline__ unsigned long long ordered_bits(double x) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | (1ull << 63));
}

struct SolveOut {
    int status;
    double d2;
    int pivots;        // simplex pivots taken
    int bland_pivots;  // of which under Bland's rule
};

// Solve the LP of one oriented pair with the G lanes of this group.  On
// return every lane holds the same SolveOut; N holds the optimal basis tree
// and potentials (valid when status == kOk).
// With `costs_set` the caller has already put the pair's costs into N (the
// register row, +inf beyond the support, oriented like the pair);
// otherwise costs come from the points.
//
// GIVEN: the costs are the caller's FP64 matrix `gcost` instead of points:
// row l, column j of the oriented pair is gcost[l * grs + j * gcs].  Such
// costs may be negative, so the tolerance scales with max |C| and the
// least-cost start orders costs by an order-preserving integer key.
template <int G, int GS, bool LT, typename TIn, int START, typename TileT, bool GIVEN = false>
__device__ __forceinline__ SolveOut solve_pair(GroupMem<G, GS> &M, TileT &tile, NodeState<G, GS, LT> &N,
                                               const PairView &pv, int d, const KOpts &o, int l, int gbase,
                                               const double *gcost = nullptr, int64_t grs = 0, int64_t gcs = 0,
                                               bool costs_set = false) {
    SolveOut out{kOk, __builtin_nan(""), 0, 0};
    const int T = pv.T, S = pv.S;
    if (T < 1 || S < 1 || T > G || S > GS) { out.status = kTooLarge; return out; }
    const bool hasR = l < T, hasC = l < S;

    // Weights: validated, then divided by their sum taken in index order.
    double pr = hasR ? ldw<TIn>(pv.wr, l) : 0.0;
    double pc = hasC ? ldw<TIn>(pv.wc, l) : 0.0;
    const bool badw = (hasR && !(isfinite(pr) && pr >= 0.0)) || (hasC && !(isfinite(pc) && pc >= 0.0));
    M.u.init.pw[l] = pr;
    if (l < GS) M.u.init.qw[l] = pc;
    wsync();
    // Loops over rows or columns stop at the largest support in the wave
    // (wave-uniform, so they branch on the scalar unit); cells beyond a
    // pair's own support hold +inf or zero and change nothing.
    const int Tw = wave_max<G>(T);
    const int Sw = wave_max<G>(S);
    double sumr = 0.0, sumc = 0.0;
#pragma unroll 4
    for (int a = 0; a < Tw; ++a) sumr += M.u.init.pw[a];   // zeros beyond the support add nothing
#pragma unroll 4
    for (int b = 0; b < Sw; ++b) sumc += M.u.init.qw[b];
    const bool badsum = !(sumr > 0.0) || !(sumc > 0.0) || !isfinite(sumr) || !isfinite(sumc);
    if (group_bits<G>(badw || badsum, gbase) != 0ull) { out.status = kBadWeights; return out; }
    pr = pr / sumr;
    pc = pc / sumc;

    // Cost row l, direct form: C_lj = sum_k (x_lk - y_jk)^2, k ascending.
    // Lane l holds row point l; column points pass through LDS, KC
    // coordinates at a time, widened to FP64 once by the lane that owns the
    // column and read back by every row lane as a broadcast.  The narrow
    // shapes accumulate straight into the register row; the LDS-tile shape
    // goes in blocks of 16 columns.
    if constexpr (GIVEN) {
#pragma unroll
        for (int j = 0; j < GS; ++j) {
            const double c = (hasR && j < S) ? gcost[(int64_t)l * grs + (int64_t)j * gcs] : INFINITY;
            put_cost<G, GS, LT>(N, tile, l, j, c);
        }
    } else if (costs_set) {
        // already in N
    } else {
        const TIn *xr = (const TIn *)pv.xr + (int64_t)l * d;
        const TIn *yc = (const TIn *)pv.xc + (int64_t)l * d;
        constexpr int KC = stage_k<G>();
        constexpr int JB = LT ? 16 : GS;
        static_for<0, GS / JB>([&](auto bc) {
            constexpr int jb = decltype(bc)::value * JB;
            double accl[LT ? JB : 1];
            auto acc = [&](auto jc) -> double & {
                if constexpr (LT) return accl[decltype(jc)::value];
                else return N.crow[jb + decltype(jc)::value];
            };
            if (jb < Sw) {
                static_for<0, JB>([&](auto jc) { acc(jc) = 0.0; });
                // The next round's coordinates are loaded while this round
                // computes (kept in the input type until used).
                TIn xn[KC], yn[KC];
#pragma unroll
                for (int q = 0; q < KC; ++q) {
                    const bool in = q < d;
                    xn[q] = (hasR && in) ? xr[q] : (TIn)0;
                    yn[q] = (hasC && in) ? yc[q] : (TIn)0;
                }
                for (int k0 = 0; k0 < d; k0 += KC) {
                    double xd[KC];
#pragma unroll
                    for (int q = 0; q < KC; ++q) {
                        xd[q] = (double)xn[q];
                        if (hasC) M.u.stage.y[l][q] = (double)yn[q];
                    }
                    if (k0 + KC < d) {
#pragma unroll
                        for (int q = 0; q < KC; ++q) {
                            const bool in = k0 + KC + q < d;
                            xn[q] = (hasR && in) ? xr[k0 + KC + q] : (TIn)0;
                            yn[q] = (hasC && in) ? yc[k0 + KC + q] : (TIn)0;
                        }
                    }
                    wsync();
                    static_for<0, JB>([&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        if (jb + j < Sw) {
                            double yv[KC];
#pragma unroll
                            for (int q = 0; q < KC; q += 2) {
                                const double2 t = *(const double2 *)&M.u.stage.y[jb + j][q];
                                yv[q] = t.x;
                                yv[q + 1] = t.y;
                            }
#pragma unroll
                            for (int q = 0; q < KC; ++q) {
                                if (k0 + q < d) {
                                    const double diff = xd[q] - yv[q];
                                    acc(jc) = fma(diff, diff, acc(jc));
                                }
                            }
                        }
                    });
                    wsync();
                }
                static_for<0, JB>([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    const double c = (hasR && jb + j < S) ? acc(jc) : INFINITY;
                    put_cost<G, GS, LT>(N, tile, l, jb + j, c);
                });
            } else {
#pragma unroll
                for (int j = 0; j < JB; ++j) {
                    put_cost<G, GS, LT>(N, tile, l, jb + j, INFINITY);
                }
            }
        });
    }
    double cmax = 0.0;
    bool finite = true;
    up_to<GS, GS / 4>(Sw, [&](auto nc) {
#pragma unroll
        for (int j = 0; j < decltype(nc)::value; ++j) {
            const bool live = hasR && j < S;
            const double c = cost_at<G, GS, LT>(N, tile, l, j);
            finite = finite & (!live | isfinite(c));
            cmax = live ? fmax(cmax, GIVEN ? fabs(c) : c) : cmax;
        }
    });
    if (group_bits<G>(!finite, gbase) != 0ull) { out.status = kBadPoints; return out; }
    cmax = group_max<G>(cmax);
    const double delta = o.tol * cmax;

    // Starting basis: t+s-1 cells forming a spanning tree.
    N.parR = -1; N.parC = -1;
    N.flowR = 0.0; N.flowC = 0.0; N.cparR = 0.0; N.cparC = 0.0;
    wsync();
    if constexpr (START == kStartLCM) {
        // Least-cost start, many cells per round.  Every open row proposes
        // its cheapest open cell; for each column the cheapest proposal wins
        // (ties: lowest row).  The winners share no row and no column, so
        // they are filled together, each with all that its row or column has
        // left, closing that line (the row when both run out).  A round that
        // would close every open row or every open column takes only the
        // cheapest proposal.  When one row (column) is left open it takes the
        // remaining columns (rows) and becomes the root.  Rows rescan only
        // when their cheapest column closes.
        using LMask = typename std::conditional<(G <= 32 && GS <= 32), uint32_t, uint64_t>::type;
        M.u.lcm.remR[l] = pr;
        if (l < GS) M.u.lcm.remC[l] = pc;
        LMask rowon = (LMask)((T == 64) ? ~0ull : ((1ull << T) - 1ull));
        LMask colon = (LMask)((S == 64) ? ~0ull : ((1ull << S) - 1ull));
        double m1 = INFINITY;
        int j1 = 0;
        up_to<GS, GS / 4>(Sw, [&](auto nc) {
#pragma unroll
            for (int j = 0; j < decltype(nc)::value; ++j) {   // +inf beyond the support
                const double c = cost_at<G, GS, LT>(N, tile, l, j);
                const bool lt = c < m1;
                m1 = lt ? c : m1;
                j1 = lt ? j : j1;
            }
        });
        // Every round closes at least one line, so T + S - 2 rounds suffice;
        // the bound makes termination unconditional.
        int rounds = 0;
#pragma unroll 1
        for (;;) {
            if (++rounds > T + S) { out.status = kInternal; return out; }
            const int nr = __popcll((uint64_t)rowon), nc = __popcll((uint64_t)colon);
            if (nr == 1) {
                const int a = __ffsll((long long)(uint64_t)rowon) - 1;
                if (l == a) {
#pragma unroll
                    for (int j = 0; j < GS; ++j)
                        if (j < Sw) M.u.lcm.lastrow[j] = cost_at<G, GS, LT>(N, tile, l, j);
                }
                wsync();
                if (hasC && ((colon >> l) & 1u)) {
                    N.parC = a; N.flowC = M.u.lcm.remC[l]; N.cparC = M.u.lcm.lastrow[l];
                }
                break;
            }
            if (nc == 1) {
                const int b = __ffsll((long long)(uint64_t)colon) - 1;
                if (hasR && ((rowon >> l) & 1u)) {
                    N.parR = b; N.flowR = M.u.lcm.remR[l]; N.cparR = cost_pick<G, GS, LT>(N, tile, l, b);
                }
                break;
            }
            const bool open = hasR && ((rowon >> l) & 1u);
            // Proposal key: the cost's bits (non-negative doubles order as
            // integers; given costs of either sign through an
            // order-preserving map) with the row in the low 6 bits, so one
            // 64-bit minimum per column picks the cheapest, then the lowest
            // row.
            const unsigned long long key =
                ((GIVEN ? ordered_bits(m1) : (unsigned long long)__double_as_longlong(m1)) & ~63ull) |
                (unsigned long long)l;
            if (l < GS) { M.u.lcm.key[l] = ~0ull; M.u.lcm.row[l] = -1; }
            if (l == 0) M.u.lcm.gkey = ~0ull;
            wsync();
            if (open) atomicMin(&M.u.lcm.key[j1], key);
            wsync();
            bool won = open && M.u.lcm.key[j1] == key;
            const double ra = M.u.lcm.remR[l], rb = M.u.lcm.remC[j1];
            const bool closeRow = ra <= rb;
            const int rclose = __popcll(group_bits<G>(won && closeRow, gbase));
            const int cclose = __popcll(group_bits<G>(won && !closeRow, gbase));
            if (rclose >= nr || cclose >= nc) {
                // only the cheapest proposal this round: an exact integer
                // minimum over the keys, which are distinct (they hold the row)
                if (open) atomicMin(&M.u.lcm.gkey, key);
                wsync();
                won = open && M.u.lcm.gkey == key;
            }
            const double x = ra < rb ? ra : rb;
            wsync();
            if (won) {
                // the only winner of row l and of column j1 this round
                M.u.lcm.remR[l] = ra - x;
                M.u.lcm.remC[j1] = rb - x;
                if (closeRow) { N.parR = j1; N.flowR = x; N.cparR = m1; }
                M.u.lcm.row[j1] = l;
                M.u.lcm.x[j1] = x;
                M.u.lcm.cost[j1] = m1;
                M.u.lcm.shut[j1] = closeRow ? 0 : 1;
            }
            const LMask rshut = (LMask)group_bits<G>(won && closeRow, gbase);
            wsync();
            const bool cdone = hasC && l < GS && M.u.lcm.row[l] >= 0 && M.u.lcm.shut[l];
            if (cdone) { N.parC = M.u.lcm.row[l]; N.flowC = M.u.lcm.x[l]; N.cparC = M.u.lcm.cost[l]; }
            const LMask cshut = (LMask)group_bits<G>(cdone, gbase);
            rowon &= ~rshut;
            colon &= ~cshut;
            wsync();
            if (hasR && ((rowon >> l) & 1u) && ((cshut >> j1) & 1u)) {
                m1 = INFINITY;
                j1 = 0;
                up_to<GS, GS / 4>(Sw, [&](auto nc) {
#pragma unroll
                    for (int j = 0; j < decltype(nc)::value; ++j) {
                        const bool lt = ((colon >> j) & 1u) && cost_at<G, GS, LT>(N, tile, l, j) < m1;
                        m1 = lt ? cost_at<G, GS, LT>(N, tile, l, j) : m1;
                        j1 = lt ? j : j1;
                    }
                });
            }
        }
        wsync();
        if (l < GS) M.u.init.colpar[l] = hasC ? N.parC : -1;
        wsync();
        N.bas = (hasR && N.parR >= 0) ? (1ull << N.parR) : 0u;
#pragma unroll
        for (int c = 0; c < GS; ++c)
            if (c < Sw && hasR && c < S && M.u.init.colpar[c] == l) N.bas |= (decltype(N.bas))1 << c;
        wsync();
        tree_jump<G, GS, LT, true>(M, N, l, T, S);
    } else if constexpr (START == kStartVogel) {
        // Vogel: close, one per round, the line whose two cheapest open cells
        // differ most (ties: rows first, lower index), filling its cheapest
        // open cell; the last open row (column) takes every open column's
        // remaining demand (row's remaining supply) and becomes the root.
        M.u.init.pw[l] = pr;
        if (l < GS) M.u.init.qw[l] = pc;
        if constexpr (!LT) {
#pragma unroll
            for (int j = 0; j < GS; ++j) tile.C[j][l] = N.crow[j];
        }
        wsync();
        uint64_t rowon = (T == 64) ? ~0ull : ((1ull << T) - 1ull);
        uint64_t colon = (S == 64) ? ~0ull : ((1ull << S) - 1ull);
#pragma unroll 1
        for (;;) {
            const int nr = __popcll(rowon), nc = __popcll(colon);
            if (nr == 1) {
                const int a = __ffsll((long long)rowon) - 1;
                if (hasC && ((colon >> l) & 1ull)) {
                    N.parC = a; N.flowC = M.u.init.qw[l]; N.cparC = tile.C[l][a];
                }
                break;
            }
            if (nc == 1) {
                const int b = __ffsll((long long)colon) - 1;
                if (hasR && ((rowon >> l) & 1ull)) {
                    N.parR = b; N.flowR = M.u.init.pw[l]; N.cparR = tile.C[b][l];
                }
                break;
            }
            double pen = -1.0;
            int key = kNoKey, other = -1;
            if (hasR && ((rowon >> l) & 1ull)) {
                double m1 = INFINITY, m2 = INFINITY;
                int j1 = -1;
                for (int j = 0; j < S; ++j) {
                    if (!((colon >> j) & 1ull)) continue;
                    const double c = tile.C[j][l];
                    if (c < m1) { m2 = m1; m1 = c; j1 = j; }
                    else if (c < m2) m2 = c;
                }
                pen = m2 - m1; key = l; other = j1;
            }
            if (hasC && ((colon >> l) & 1ull)) {
                double m1 = INFINITY, m2 = INFINITY;
                int i1 = -1;
                for (int a = 0; a < T; ++a) {
                    if (!((rowon >> a) & 1ull)) continue;
                    const double c = tile.C[l][a];
                    if (c < m1) { m2 = m1; m1 = c; i1 = a; }
                    else if (c < m2) m2 = c;
                }
                const double pc2 = m2 - m1;
                if (pc2 > pen) { pen = pc2; key = 64 + l; other = i1; }
            }
            double npen = key == kNoKey ? INFINITY : -pen;
            int packed = key == kNoKey ? kNoKey : key * 128 + other;
            group_argmin<G>(npen, packed);
            const int bkey = packed >> 7, bother = packed & 127;
            const int a = bkey < 64 ? bkey : bother;
            const int b = bkey < 64 ? bother : bkey - 64;
            double ra = M.u.init.pw[a], rb = M.u.init.qw[b];
            const double x = ra < rb ? ra : rb;
            ra -= x;
            rb -= x;
            wsync();
            if (l == 0) { M.u.init.pw[a] = ra; M.u.init.qw[b] = rb; }
            if (ra <= rb) {
                if (l == a) { N.parR = b; N.flowR = x; N.cparR = tile.C[b][a]; }
                rowon &= ~(1ull << a);
            } else {
                if (l == b) { N.parC = a; N.flowC = x; N.cparC = tile.C[b][a]; }
                colon &= ~(1ull << b);
            }
            wsync();
        }
        wsync();
        if (l < GS) M.u.init.colpar[l] = hasC ? N.parC : -1;
        wsync();
        N.bas = (hasR && N.parR >= 0) ? (1ull << N.parR) : 0u;
#pragma unroll
        for (int c = 0; c < GS; ++c)
            if (c < Sw && hasR && c < S && M.u.init.colpar[c] == l) N.bas |= (decltype(N.bas))1 << c;
        wsync();
        tree_jump<G, GS, LT, true>(M, N, l, T, S);
    } else {
        // North-west corner, all nodes at once.  With inclusive prefix sums
        // P_a of p and Q_b of q, the corner walk moves down after row a when
        // P_a <= Q_b for the current column b (ties: down first).  So row a
        // (a >= 1) hangs below column #{b <= S-2 : Q_b < P_{a-1}} and column b
        // (b >= 1) below row #{a <= T-2 : P_a <= Q_{b-1}}; a cell's flow is the
        // overlap of its row and column intervals, the last row and column
        // extending to max(P_{T-1}, Q_{S-1}).  Row 0 is the root.
        M.u.init.pw[l] = pr;
        if (l < GS) M.u.init.qw[l] = pc;
        wsync();
        double Pl = 0.0, Ql = 0.0;
#pragma unroll 4
        for (int a = 0; a < Tw; ++a) Pl += (a <= l) ? M.u.init.pw[a] : 0.0;
#pragma unroll 4
        for (int b = 0; b < Sw; ++b) Ql += (b <= l) ? M.u.init.qw[b] : 0.0;
        M.u.init.P[l] = Pl;
        if (l < GS) M.u.init.Q[l] = Ql;
        wsync();
        const double END = fmax(M.u.init.P[T - 1], M.u.init.Q[S - 1]);
        int idxR = 0x3fffffff, idxC = 0x3fffffff;
        if (hasR && l >= 1) {
            const double start = M.u.init.P[l - 1];
            int b = 0;
#pragma unroll 4
            for (int j = 0; j < Sw - 1; ++j) {
                const double qb = M.u.init.Q[j];
                b += (j <= S - 2 && qb < start) ? 1 : 0;
            }
            const double er = (l == T - 1) ? END : Pl;
            const double ec = (b == S - 1) ? END : M.u.init.Q[b];
            N.parR = b;
            N.flowR = fmin(er, ec) - start;
            N.cparR = cost_pick<G, GS, LT>(N, tile, l, b);
            idxR = l + b + 1;
        } else if (hasR) {
            idxR = 0;
        }
        if (hasC) {
            double start = 0.0;
            int a = 0;
            if (l >= 1) {
                start = M.u.init.Q[l - 1];
#pragma unroll 4
                for (int i = 0; i < Tw - 1; ++i) {
                    const double pa = M.u.init.P[i];
                    a += (i <= T - 2 && pa <= start) ? 1 : 0;
                }
            }
            const double ec = (l == S - 1) ? END : Ql;
            const double er = (a == T - 1) ? END : M.u.init.P[a];
            N.parC = a;
            N.flowC = fmin(er, ec) - start;
            idxC = l + a + 1;
        }
        // The walk's node sequence splits into runs of rows and runs of
        // columns; a node hangs below the last node of the run before its
        // own, so its ancestors are itself plus every run's last node visited
        // before it.
        if (l < GS) M.u.init.colpar[l] = hasC ? N.parC : -1;
        if (hasR) M.u.init.kind[idxR] = 0;
        if (hasC) M.u.init.kind[idxC] = 1;
        wsync();
        // Basic cells of row l and the parent-edge costs of its child columns.
        N.bas = (hasR && N.parR >= 0) ? (1ull << N.parR) : 0u;
#pragma unroll
        for (int c = 0; c < GS; ++c) {
            if (c < Sw && hasR && c < S && M.u.init.colpar[c] == l) {
                N.bas |= (decltype(N.bas))1 << c;
                M.u.init.colcpar[c] = cost_at<G, GS, LT>(N, tile, l, c);
            }
        }
        const int lastpos = T + S - 1;
        const int nR = idxR + 1 < 2 * G ? idxR + 1 : 2 * G - 1;
        const int nC = idxC + 1 < 2 * G ? idxC + 1 : 2 * G - 1;
        const bool lastR = hasR && (idxR == lastpos || M.u.init.kind[nR] != 0);
        const bool lastC = hasC && (idxC == lastpos || M.u.init.kind[nC] != 1);
        M.u.init.lastpos[l] = lastR ? idxR : 0x3fffffff;
        M.u.init.lastpos[G + l] = lastC ? idxC : 0x3fffffff;
        wsync();
        Mask<G> aR = Mask<G>::node(l), aC = Mask<G>::node(G + l);
#pragma unroll 4
        for (int n = 0; n < Tw; ++n) {
            const int lp = M.u.init.lastpos[n];
            if (lp < idxR) aR = aR | Mask<G>::node(n);
            if (lp < idxC) aC = aC | Mask<G>::node(n);
        }
#pragma unroll 4
        for (int n = G; n < G + Sw; ++n) {
            const int lp = M.u.init.lastpos[n];
            if (lp < idxR) aR = aR | Mask<G>::node(n);
            if (lp < idxC) aC = aC | Mask<G>::node(n);
        }
        N.ancR = hasR ? aR : Mask<G>::none();
        N.ancC = hasC ? aC : Mask<G>::none();
        if (hasC) N.cparC = M.u.init.colcpar[l];
        wsync();
        tree_jump<G, GS, LT, false>(M, N, l, T, S);
    }

    const long long cap = o.max_pivots > 0 ? (long long)o.max_pivots
                                           : (50LL * T * S > 100 ? 50LL * T * S : 100LL);
    long long pivots = 0;
    int degenerate_run = 0, bland_pivots = 0;
    const int bland_after = o.bland_after > 0 ? o.bland_after : 2 * (T + S);
    bool bland = false, fresh = true;
#pragma unroll 1
    for (;;) {
        // Pricing: most negative reduced cost (Bland: first negative cell).
        // Padding cells hold +inf, so every lane runs the same loop.
        double best = -delta, bestC = 0.0;
        int bj = -1;   // column of the lane's best cell (the key is formed after the loop)
        const double u = N.potR;
        // Columns go in chunks of PC so that their loads are in flight
        // together; the 64-lane shapes run few waves per SIMD and need the
        // widest chunks to hide the LDS latency (measured: 8 / 4 / 2).
        constexpr int PC = LT ? 8 : (G == 64 ? 4 : 2);
        if (!bland) {
#pragma unroll
            for (int j0 = 0; j0 < GS; j0 += PC) {
                if (j0 < Sw) {
                    double cc[PC], vv[PC];
#pragma unroll
                    for (int q = 0; q < PC; ++q) {
                        cc[q] = cost_at<G, GS, LT>(N, tile, l, j0 + q);
                        vv[q] = M.vpot[j0 + q];
                    }
#pragma unroll
                    for (int q = 0; q < PC; ++q) {
                        const int j = j0 + q;
                        const double r = (cc[q] - u) - vv[q];
                        const bool cand = (((N.bas >> j) & 1u) == 0u) & (r < best);
                        best = cand ? r : best;
                        bestC = cand ? cc[q] : bestC;
                        bj = cand ? j : bj;
                    }
                }
            }
        } else {
#pragma unroll
            for (int j0 = GS - PC; j0 >= 0; j0 -= PC) {
                if (j0 < Sw) {
                    double cc[PC], vv[PC];
#pragma unroll
                    for (int q = 0; q < PC; ++q) {
                        cc[q] = cost_at<G, GS, LT>(N, tile, l, j0 + q);
                        vv[q] = M.vpot[j0 + q];
                    }
#pragma unroll
                    for (int q = PC - 1; q >= 0; --q) {
                        const int j = j0 + q;
                        const double r = (cc[q] - u) - vv[q];
                        const bool cand = (((N.bas >> j) & 1u) == 0u) & (r < -delta);
                        best = cand ? r : best;
                        bestC = cand ? cc[q] : bestC;
                        bj = cand ? j : bj;
                    }
                }
            }
        }
        double key = bland ? 0.0 : best;
        int kidx = bj >= 0 ? l * 64 + bj : kNoKey;
        group_argmin<G>(key, kidx);
        if (kidx == kNoKey) {
            if (fresh) break;
            // Recompute the potentials from the tree before concluding.
            tree_jump<G, GS, LT, false>(M, N, l, T, S);
            fresh = true;
            continue;
        }
        if (pivots >= cap) {
            out.status = kPivotCap;
            out.pivots = (int)pivots;
            out.bland_pivots = bland_pivots;
            return out;
        }
        const int er = kidx >> 6, ec = kidx & 63;
        if (l == er) { M.bc_r = best; M.bc_c = bestC; }
        wsync();
        const double re = M.bc_r, Ce = M.bc_c;
        const Mask<G> Ar = M.ancRm[er];
        const Mask<G> Ac = M.ancCm[ec];
        // Edges whose flow decreases: rows on the entering row's side of the
        // path, columns on the entering column's side.
        const Mask<G> onR = Ar.andnot(Ac), onC = Ac.andnot(Ar);
        const Mask<G> minus = (onR & Mask<G>::rows_only()) | (onC & Mask<G>::cols_only());
        const Mask<G> plus = (onR & Mask<G>::cols_only()) | (onC & Mask<G>::rows_only());
        // Ratio test: least flow on a decreasing edge, ties to the lowest cell.
        double th = INFINITY;
        int tkey = kNoKey;
        const bool mR = hasR && minus.has(l), mC = hasC && minus.has(G + l);
        th = mR ? N.flowR : th;
        tkey = mR ? (l * 64 + N.parR) * 256 + l : tkey;
        {
            const int k2 = (N.parC * 64 + l) * 256 + (G + l);
            const bool takeC = mC & ((N.flowC < th) | ((N.flowC == th) & (k2 < tkey)));
            th = takeC ? N.flowC : th;
            tkey = takeC ? k2 : tkey;
        }
        group_argmin<G>(th, tkey);
        const double theta = th;
        const int Lnode = tkey & 255;
        const int lcell = tkey >> 8, lr = lcell >> 6, lc = lcell & 63;
        N.flowR += mR ? -theta : ((hasR & plus.has(l)) ? theta : 0.0);
        N.flowC += mC ? -theta : ((hasC & plus.has(G + l)) ? theta : 0.0);
        // Subtree cut off by the leaving edge, and the entering end inside it.
        const bool inR = hasR && N.ancR.has(Lnode);
        const bool inC = hasC && N.ancC.has(Lnode);
        const Mask<G> Sub = Mask<G>::from_bits(group_bits<G>(inR, gbase), group_bits<G>(inC, gbase));
        const bool q_is_row = Sub.has(er);
        const int qnode = q_is_row ? er : G + ec;
        const Mask<G> Ap = q_is_row ? Ac : Ar;
        const Mask<G> stem = (q_is_row ? Ar : Ac) & Sub;
        const double dU = q_is_row ? re : -re;
        const double dV = -dU;
        const bool stR = hasR && stem.has(l), stC = hasC && stem.has(G + l);
        // Scatter for re-hanging: each stem node except L tells its parent
        // who its new parent is, and hands over the edge's flow and cost.
        if (stR && l != Lnode) {
            M.u.piv.newpar[G + N.parR] = l;
            M.u.piv.newflow[G + N.parR] = N.flowR;
            M.u.piv.newcpar[G + N.parR] = N.cparR;
        }
        if (stC && G + l != Lnode) {
            M.u.piv.newpar[N.parC] = G + l;
            M.u.piv.newflow[N.parC] = N.flowC;
            M.u.piv.newcpar[N.parC] = N.cparC;
        }
        if (stR) M.u.piv.stemtab[(N.ancR & stem).popc() - 1] = l;
        if (stC) M.u.piv.stemtab[(N.ancC & stem).popc() - 1] = G + l;
        wsync();
        if (inR) {
            const Mask<G> A = N.ancR & Sub;
            const int y = M.u.piv.stemtab[(A & stem).popc() - 1];
            N.ancR = Ap | (A ^ stem) | Mask<G>::node(y);
            N.potR += dU;
            M.ancRm[l] = N.ancR;
        }
        if (inC) {
            const Mask<G> A = N.ancC & Sub;
            const int y = M.u.piv.stemtab[(A & stem).popc() - 1];
            N.ancC = Ap | (A ^ stem) | Mask<G>::node(y);
            N.potC += dV;
            M.ancCm[l] = N.ancC;
            M.vpot[l] = N.potC;
        }
        if (stR) {
            if (l == qnode) { N.parR = ec; N.flowR = theta; N.cparR = Ce; }
            else {
                N.parR = M.u.piv.newpar[l] - G;
                N.flowR = M.u.piv.newflow[l];
                N.cparR = M.u.piv.newcpar[l];
            }
        }
        if (stC) {
            if (G + l == qnode) { N.parC = er; N.flowC = theta; N.cparC = Ce; }
            else {
                N.parC = M.u.piv.newpar[G + l];
                N.flowC = M.u.piv.newflow[G + l];
                N.cparC = M.u.piv.newcpar[G + l];
            }
        }
        if (l == er) N.bas |= (decltype(N.bas))1 << ec;
        if (l == lr) N.bas &= ~((decltype(N.bas))1 << lc);
        wsync();
        ++pivots;
        bland_pivots += bland ? 1 : 0;
        fresh = false;
        if (theta == 0.0) {
            if (++degenerate_run >= bland_after) bland = true;
        } else {
            degenerate_run = 0;
            bland = false;
        }
    }

    // Objective: sum over tree edges of flow * cost, in node-index order.
    M.u.fin.obj[l] = (hasR && N.parR >= 0) ? N.flowR * N.cparR : 0.0;
    M.u.fin.obj[G + l] = (hasC && N.parC >= 0) ? N.flowC * N.cparC : 0.0;
    wsync();
    double sum = 0.0;
#pragma unroll 4
    for (int n = 0; n < Tw; ++n) sum += M.u.fin.obj[n];
#pragma unroll 4
    for (int n = G; n < G + Sw; ++n) sum += M.u.fin.obj[n];
    out.d2 = o.want_sqrt ? sqrt(sum) : sum;
    out.pivots = (int)pivots;
    out.bland_pivots = bland_pivots;
    wsync();
    return out;
}

// Dense plan (caller's orientation) and duals of a solved pair.
template <int G, int GS, bool LT>
__device__ __forceinline__ void write_certificate(GroupMem<G, GS> &M, const NodeState<G, GS, LT> &N,
                                                  const PairView &pv, int l, double *plan, double *duals) {
    const int T = pv.T, S = pv.S;
    const bool hasR = l < T, hasC = l < S;
    if (l < GS) {
        M.u.fin.colflow[l] = hasC ? N.flowC : 0.0;
        M.u.fin.colpar[l] = hasC ? N.parC : -1;
    }
    wsync();
    if (plan && hasR) {
        for (int j = 0; j < S; ++j) {
            double w = 0.0;
            if (N.parR == j) w = N.flowR;
            else if (M.u.fin.colpar[j] == l) w = M.u.fin.colflow[j];
            // caller's frame: A side is t x s; rows here are A unless swapped
            const int64_t idx = pv.swapped ? ((int64_t)j * T + l) : ((int64_t)l * S + j);
            plan[idx] = w;
        }
    }
    if (duals) {
        const int tA = pv.swapped ? S : T;   // u (A side) then v (B side)
        if (!pv.swapped) {
            if (hasR) duals[l] = N.potR;
            if (hasC) duals[tA + l] = N.potC;
        } else {
            if (hasC) duals[l] = N.potC;
            if (hasR) duals[tA + l] = N.potR;
        }
    }
    wsync();
}

}  // namespace d2
