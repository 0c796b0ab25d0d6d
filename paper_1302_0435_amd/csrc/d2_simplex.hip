// Wave-parallel transportation simplex for the squared Mallows distance.
//
// One pair (P, Q) is the LP of Eq. (1) with the centroid fixed (paper,
// Sec. 1.1): minimise sum_ab w_ab |x_a - y_b|^2 over w >= 0 with row sums p
// and column sums q.  The paper leaves the LP solver open; this file solves
// it with the transportation simplex (u-v method): a starting basis (north-
// west corner or Vogel), dual potentials u, v with u_a + v_b = C_ab on the
// basis, pricing r_ab = C_ab - u_a - v_b, and pivots around the cycle that
// the entering cell closes in the basis spanning tree.
//
// GPU mapping.  A "group" of G lanes (G = 16, 32 or 64, so 64/G pairs per
// wavefront) owns one pair at a time.  The pair is oriented so that rows are
// the larger support (D^2 is symmetric).  Lane l owns row node l and column
// node l of the basis tree.  Every node stores its parent, the flow and cost
// of the edge to its parent, its potential and its ancestor set as a bitmask
// over the 2G nodes.  With ancestor masks a pivot needs no pointer chasing:
//   * the cycle of entering cell (r, c) is the tree path r..c, i.e. the nodes
//     in anc(r) xor anc(c); the edges whose flow decreases are the row nodes
//     on r's side and the column nodes on c's side;
//   * the ratio test is a group min-reduction over those edges' flows;
//   * the subtree cut off by the leaving edge is {x : L in anc(x)}, found by
//     one ballot; it is re-hung below the entering cell, the edges on the
//     path from the entering end up to L ("stem") change direction, and the
//     new ancestor set of every moved node is anc(p) | (A xor stem) | {y},
//     where A is its old ancestor set inside the subtree and y its deepest
//     ancestor on the stem (looked up by position along the stem);
//   * potentials change only inside the moved subtree, by +-r_entering.
// Potentials are recomputed from the tree by pointer jumping at the start
// and once more before declaring optimality, so rounding drift in the
// incremental updates cannot end the solve early.
//
// All arithmetic that decides the result uses fixed orders that do not
// depend on G (serial index-order sums, exact min/max reductions), so every
// group width returns the same bits for the same pair.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "d2_internal.h"

namespace d2 {

enum { kOk = 0, kBadWeights = 1, kTooLarge = 2, kPivotCap = 3, kBadPoints = 4 };

// ------------------------------------------------------------------ masks

// Node sets of one group's tree.  G <= 32: rows in bits [0,32), columns in
// bits [32,64) of one word.  G = 64: one word each.
template <int G>
struct Mask {
    uint64_t m;
    __device__ static Mask none() { return {0ull}; }
    __device__ static Mask row(int i) { return {1ull << i}; }
    __device__ static Mask col(int j) { return {1ull << (32 + j)}; }
    __device__ static Mask node(int id) { return id < G ? row(id) : col(id - G); }
    __device__ static Mask rows_only() { return {0x00000000FFFFFFFFull}; }
    __device__ static Mask cols_only() { return {0xFFFFFFFF00000000ull}; }
    __device__ static Mask from_bits(uint64_t r, uint64_t c) { return {r | (c << 32)}; }
    __device__ Mask operator|(Mask o) const { return {m | o.m}; }
    __device__ Mask operator&(Mask o) const { return {m & o.m}; }
    __device__ Mask operator^(Mask o) const { return {m ^ o.m}; }
    __device__ Mask andnot(Mask o) const { return {m & ~o.m}; }
    __device__ bool has(int id) const { return id < G ? ((m >> id) & 1ull) : ((m >> (32 + id - G)) & 1ull); }
    __device__ bool has_row(int i) const { return (m >> i) & 1ull; }
    __device__ int popc() const { return __popcll(m); }
    __device__ Mask bcast(int src) const { return {__shfl(m, src, G)}; }
};

template <>
struct Mask<64> {
    uint64_t r, c;
    __device__ static Mask none() { return {0ull, 0ull}; }
    __device__ static Mask row(int i) { return {1ull << i, 0ull}; }
    __device__ static Mask col(int j) { return {0ull, 1ull << j}; }
    __device__ static Mask node(int id) { return id < 64 ? row(id) : col(id - 64); }
    __device__ static Mask rows_only() { return {~0ull, 0ull}; }
    __device__ static Mask cols_only() { return {0ull, ~0ull}; }
    __device__ static Mask from_bits(uint64_t rr, uint64_t cc) { return {rr, cc}; }
    __device__ Mask operator|(Mask o) const { return {r | o.r, c | o.c}; }
    __device__ Mask operator&(Mask o) const { return {r & o.r, c & o.c}; }
    __device__ Mask operator^(Mask o) const { return {r ^ o.r, c ^ o.c}; }
    __device__ Mask andnot(Mask o) const { return {r & ~o.r, c & ~o.c}; }
    __device__ bool has(int id) const { return id < 64 ? ((r >> id) & 1ull) : ((c >> (id - 64)) & 1ull); }
    __device__ bool has_row(int i) const { return (r >> i) & 1ull; }
    __device__ int popc() const { return __popcll(r) + __popcll(c); }
    __device__ Mask bcast(int src) const { return {__shfl(r, src, 64), __shfl(c, src, 64)}; }
};

template <int G>
struct Log2 { static constexpr int v = G == 16 ? 4 : (G == 32 ? 5 : 6); };

// Orders LDS traffic between lanes of one wavefront (hardware executes a
// wavefront's LDS operations in order; this keeps the compiler from moving
// loads above stores).
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------ group memory

template <int G>
struct GroupMem {
    double C[G][G + 1];  // cost tile, rows x columns (padded stride)
    double vpot[G];      // column potentials, read by every row lane when pricing
    union {
        struct { double pw[G]; double qw[G]; } w;  // weights / remaining supply and demand
        struct { int jmp[2 * G]; Mask<G> anc[2 * G]; double val[2 * G]; } jump;
        struct { int newpar[2 * G]; int stemtab[2 * G]; double newflow[2 * G]; double newcpar[2 * G]; } piv;
        struct { double obj[2 * G]; double colflow[G]; int colpar[G]; } fin;
    } u;
};

// Per-lane state: row node l and column node l.
template <int G>
struct NodeState {
    int parR, parC;          // parent index (a column / a row), -1 at the root
    double flowR, flowC;     // flow on the edge to the parent
    double cparR, cparC;     // cost of the edge to the parent
    double potR, potC;       // u_l, v_l
    Mask<G> ancR, ancC;      // ancestors including the node itself
    uint64_t bas;            // basic cells of row l, as a column bitmask
};

template <typename T>
__device__ __forceinline__ double ldw(const void *p, int64_t i) {
    return (double)((const T *)p)[i];
}

// (value, index) minimum over the group, lowest index on equal values.
template <int G>
__device__ __forceinline__ void group_argmin(double &v, int &i) {
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) {
        double ov = __shfl_xor(v, off, G);
        int oi = __shfl_xor(i, off, G);
        bool take = (ov < v) || (ov == v && oi < i);
        v = take ? ov : v;
        i = take ? oi : i;
    }
}

template <int G>
__device__ __forceinline__ double group_max(double v) {
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, G));
    return v;
}

template <int G>
__device__ __forceinline__ bool group_any(bool p, int gbase) {
    uint64_t b = __ballot(p);
    uint64_t gm = G == 64 ? ~0ull : ((1ull << G) - 1ull);
    return ((b >> gbase) & gm) != 0ull;
}

template <int G>
__device__ __forceinline__ uint64_t group_bits(bool p, int gbase) {
    uint64_t b = __ballot(p);
    uint64_t gm = G == 64 ? ~0ull : ((1ull << G) - 1ull);
    return (b >> gbase) & gm;
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

// ---------------------------------------------------------- tree rebuild

// Ancestor masks and potentials of every node from the parent pointers and
// parent-edge costs, by pointer jumping (log2(2G) rounds).  The potential of
// node x is sign(x) * sum over the path x..root of sign(n) * cpar(n) with
// sign = (-1)^depth, which unrolls u_a + v_b = C_ab along the path.
template <int G>
__device__ void rebuild_tree(GroupMem<G> &M, NodeState<G> &N, int l, int T, int S) {
    const bool hasR = l < T, hasC = l < S;
    const int idR = l, idC = G + l;
    int jR = (hasR && N.parR >= 0) ? G + N.parR : idR;
    int jC = (hasC && N.parC >= 0) ? N.parC : idC;
    Mask<G> aR = hasR ? Mask<G>::row(l) : Mask<G>::none();
    Mask<G> aC = hasC ? Mask<G>::col(l) : Mask<G>::none();
    M.u.jump.jmp[idR] = jR;
    M.u.jump.jmp[idC] = jC;
    M.u.jump.anc[idR] = aR;
    M.u.jump.anc[idC] = aC;
    wsync();
#pragma unroll 1
    for (int k = 0; k < Log2<G>::v + 1; ++k) {
        int nR = M.u.jump.jmp[jR], nC = M.u.jump.jmp[jC];
        Mask<G> xR = M.u.jump.anc[jR], xC = M.u.jump.anc[jC];
        wsync();
        aR = aR | xR;
        aC = aC | xC;
        jR = nR;
        jC = nC;
        M.u.jump.jmp[idR] = jR;
        M.u.jump.jmp[idC] = jC;
        M.u.jump.anc[idR] = aR;
        M.u.jump.anc[idC] = aC;
        wsync();
    }
    N.ancR = aR;
    N.ancC = aC;
    const double sR = ((aR.popc() - 1) & 1) ? -1.0 : 1.0;
    const double sC = ((aC.popc() - 1) & 1) ? -1.0 : 1.0;
    double vR = (hasR && N.parR >= 0) ? sR * N.cparR : 0.0;
    double vC = (hasC && N.parC >= 0) ? sC * N.cparC : 0.0;
    jR = (hasR && N.parR >= 0) ? G + N.parR : idR;
    jC = (hasC && N.parC >= 0) ? N.parC : idC;
    M.u.jump.jmp[idR] = jR;
    M.u.jump.jmp[idC] = jC;
    M.u.jump.val[idR] = vR;
    M.u.jump.val[idC] = vC;
    wsync();
#pragma unroll 1
    for (int k = 0; k < Log2<G>::v + 1; ++k) {
        int nR = M.u.jump.jmp[jR], nC = M.u.jump.jmp[jC];
        double xR = M.u.jump.val[jR], xC = M.u.jump.val[jC];
        wsync();
        vR += xR;
        vC += xC;
        jR = nR;
        jC = nC;
        M.u.jump.jmp[idR] = jR;
        M.u.jump.jmp[idC] = jC;
        M.u.jump.val[idR] = vR;
        M.u.jump.val[idC] = vC;
        wsync();
    }
    N.potR = sR * vR;
    N.potC = sC * vC;
    if (hasC) M.vpot[l] = N.potC;
    wsync();
}

// ------------------------------------------------------------ one solve

struct SolveOut {
    int status;
    double d2;
};

// Solve the LP of one oriented pair with the G lanes of this group.  On
// return every lane holds the same SolveOut; N holds the optimal basis tree
// and potentials (valid when status == kOk).
template <int G, typename TIn>
__device__ SolveOut solve_pair(GroupMem<G> &M, NodeState<G> &N, const PairView &pv, int d,
                               const KOpts &o, int l, int gbase) {
    SolveOut out{kOk, __builtin_nan("")};
    const int T = pv.T, S = pv.S;
    if (T < 1 || S < 1 || T > G || S > G) { out.status = kTooLarge; return out; }
    const bool hasR = l < T, hasC = l < S;

    // Weights: validated, then divided by their sum taken in index order.
    double pr = hasR ? ldw<TIn>(pv.wr, l) : 0.0;
    double pc = hasC ? ldw<TIn>(pv.wc, l) : 0.0;
    bool badw = (hasR && !(isfinite(pr) && pr >= 0.0)) || (hasC && !(isfinite(pc) && pc >= 0.0));
    M.u.w.pw[l] = pr;
    M.u.w.qw[l] = pc;
    wsync();
    double sumr = 0.0, sumc = 0.0;
    for (int a = 0; a < T; ++a) sumr += M.u.w.pw[a];
    for (int b = 0; b < S; ++b) sumc += M.u.w.qw[b];
    badw = badw || !(sumr > 0.0) || !(sumc > 0.0) || !isfinite(sumr) || !isfinite(sumc);
    if (group_any<G>(badw, gbase)) { out.status = kBadWeights; return out; }
    pr = pr / sumr;
    pc = pc / sumc;
    wsync();
    M.u.w.pw[l] = pr;
    M.u.w.qw[l] = pc;

    // Cost tile, direct form: C_ab = sum_k (x_ak - y_bk)^2.
    double cmax = 0.0;
    bool finite = true;
    if (hasR) {
        const TIn *xr = (const TIn *)pv.xr + (int64_t)l * d;
        for (int j = 0; j < S; ++j) {
            const TIn *yc = (const TIn *)pv.xc + (int64_t)j * d;
            double acc = 0.0;
            for (int k = 0; k < d; ++k) {
                double diff = (double)xr[k] - (double)yc[k];
                acc = fma(diff, diff, acc);
            }
            M.C[l][j] = acc;
            finite = finite && isfinite(acc);
            cmax = fmax(cmax, acc);
        }
    }
    if (group_any<G>(!finite, gbase)) { out.status = kBadPoints; return out; }
    cmax = group_max<G>(cmax);
    const double delta = o.tol * cmax;
    wsync();

    // Starting basis: t+s-1 cells forming a spanning tree.
    N.parR = -1; N.parC = -1;
    N.flowR = 0.0; N.flowC = 0.0; N.cparR = 0.0; N.cparC = 0.0;
    if (o.init == D2_INIT_VOGEL) {
        // Vogel: close, one per round, the line whose two cheapest open cells
        // differ most (ties: rows first, lower index), filling its cheapest
        // open cell; the last open row (column) takes every open column's
        // remaining demand (row's remaining supply) and becomes the root.
        uint64_t rowon = (T == 64) ? ~0ull : ((1ull << T) - 1ull);
        uint64_t colon = (S == 64) ? ~0ull : ((1ull << S) - 1ull);
#pragma unroll 1
        for (;;) {
            int nr = __popcll(rowon), nc = __popcll(colon);
            if (nr == 1) {
                int a = __ffsll((long long)rowon) - 1;
                if (hasC && ((colon >> l) & 1ull)) {
                    N.parC = a; N.flowC = M.u.w.qw[l]; N.cparC = M.C[a][l];
                }
                break;
            }
            if (nc == 1) {
                int b = __ffsll((long long)colon) - 1;
                if (hasR && ((rowon >> l) & 1ull)) {
                    N.parR = b; N.flowR = M.u.w.pw[l]; N.cparR = M.C[l][b];
                }
                break;
            }
            double pen = -1.0;
            int key = 0x7fffffff, other = -1;
            if (hasR && ((rowon >> l) & 1ull)) {
                double m1 = INFINITY, m2 = INFINITY;
                int j1 = -1;
                for (int j = 0; j < S; ++j) {
                    if (!((colon >> j) & 1ull)) continue;
                    double c = M.C[l][j];
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
                    double c = M.C[a][l];
                    if (c < m1) { m2 = m1; m1 = c; i1 = a; }
                    else if (c < m2) m2 = c;
                }
                double pc2 = m2 - m1;
                if (pc2 > pen) { pen = pc2; key = 64 + l; other = i1; }
            }
            // max penalty, then lowest key; carry `other`
            double npen = -pen;
            int packed = key * 128 + (other < 0 ? 127 : other);
            group_argmin<G>(npen, packed);
            int bkey = packed >> 7, bother = packed & 127;
            int a = bkey < 64 ? bkey : bother;
            int b = bkey < 64 ? bother : bkey - 64;
            double ra = M.u.w.pw[a], rb = M.u.w.qw[b];
            double x = ra < rb ? ra : rb;
            ra -= x;
            rb -= x;
            wsync();
            if (l == 0) { M.u.w.pw[a] = ra; M.u.w.qw[b] = rb; }
            if (ra <= rb) {
                if (l == a) { N.parR = b; N.flowR = x; N.cparR = M.C[a][b]; }
                rowon &= ~(1ull << a);
            } else {
                if (l == b) { N.parC = a; N.flowC = x; N.cparC = M.C[a][b]; }
                colon &= ~(1ull << b);
            }
            wsync();
        }
    } else {
        // North-west corner; the last row takes each remaining column's
        // demand, the last column each remaining row's supply; on a tie the
        // walk moves down and keeps a zero cell.  Row 0 is the root.
        int a = 0, b = 0, newer = G;  // first new node: column 0
        double rs = M.u.w.pw[0], rd = M.u.w.qw[0];
#pragma unroll 1
        for (;;) {
            double x = (a == T - 1) ? rd : ((b == S - 1) ? rs : (rs < rd ? rs : rd));
            double c = M.C[a][b];
            if (newer < G) {
                if (l == newer) { N.parR = b; N.flowR = x; N.cparR = c; }
            } else {
                if (l == newer - G) { N.parC = a; N.flowC = x; N.cparC = c; }
            }
            rs -= x;
            rd -= x;
            if (a == T - 1 && b == S - 1) break;
            if (a == T - 1) { b++; rd = M.u.w.qw[b]; newer = G + b; }
            else if (b == S - 1) { a++; rs = M.u.w.pw[a]; newer = a; }
            else if (rs <= rd) { a++; rs = M.u.w.pw[a]; newer = a; }
            else { b++; rd = M.u.w.qw[b]; newer = G + b; }
        }
    }
    wsync();

    // Basic cells per row: the row's own parent edge plus the columns that
    // hang below it.
    M.u.fin.colpar[l] = hasC ? N.parC : -1;
    wsync();
    N.bas = (hasR && N.parR >= 0) ? (1ull << N.parR) : 0ull;
    if (hasR)
        for (int c = 0; c < S; ++c)
            if (M.u.fin.colpar[c] == l) N.bas |= 1ull << c;
    wsync();

    rebuild_tree<G>(M, N, l, T, S);

    const long long cap = o.max_pivots > 0 ? (long long)o.max_pivots
                                           : (50LL * T * S > 100 ? 50LL * T * S : 100LL);
    long long pivots = 0;
    int degenerate_run = 0;
    bool bland = false, fresh = true;
#pragma unroll 1
    for (;;) {
        // Pricing: most negative reduced cost (Bland: first negative cell).
        double best = -delta, bestC = 0.0;
        int bidx = 0x7fffffff;
        if (hasR) {
            const double u = N.potR;
            for (int j = 0; j < S; ++j) {
                if ((N.bas >> j) & 1ull) continue;
                double c = M.C[l][j];
                double r = (c - u) - M.vpot[j];
                if (r < best) {
                    best = r; bestC = c; bidx = l * 64 + j;
                    if (bland) break;
                }
            }
        }
        double key = bland ? 0.0 : best;
        int kidx = bidx;
        group_argmin<G>(key, kidx);
        if (kidx == 0x7fffffff) {
            if (fresh) break;
            // Refresh the potentials from the tree before concluding.
            rebuild_tree<G>(M, N, l, T, S);
            fresh = true;
            continue;
        }
        if (pivots >= cap) { out.status = kPivotCap; return out; }
        const int er = kidx >> 6, ec = kidx & 63;
        const double re = __shfl(best, er, G);
        const double Ce = __shfl(bestC, er, G);
        const Mask<G> Ar = N.ancR.bcast(er);
        const Mask<G> Ac = N.ancC.bcast(ec);
        // Edges whose flow decreases: rows on the entering row's side of the
        // path, columns on the entering column's side.
        const Mask<G> onR = Ar.andnot(Ac), onC = Ac.andnot(Ar);
        const Mask<G> minus = (onR & Mask<G>::rows_only()) | (onC & Mask<G>::cols_only());
        const Mask<G> plus = (onR & Mask<G>::cols_only()) | (onC & Mask<G>::rows_only());
        // Ratio test: least flow on a decreasing edge, ties to the lowest cell.
        double th = INFINITY;
        int tkey = 0x7fffffff;
        if (hasR && minus.has(l)) { th = N.flowR; tkey = (l * 64 + N.parR) * 256 + l; }
        if (hasC && minus.has(G + l)) {
            int k2 = (N.parC * 64 + l) * 256 + (G + l);
            if (N.flowC < th || (N.flowC == th && k2 < tkey)) { th = N.flowC; tkey = k2; }
        }
        group_argmin<G>(th, tkey);
        const double theta = th;
        const int Lnode = tkey & 255;
        const int lcell = tkey >> 8, lr = lcell >> 6, lc = lcell & 63;
        if (hasR) {
            if (minus.has(l)) N.flowR -= theta;
            else if (plus.has(l)) N.flowR += theta;
        }
        if (hasC) {
            if (minus.has(G + l)) N.flowC -= theta;
            else if (plus.has(G + l)) N.flowC += theta;
        }
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
        }
        if (inC) {
            const Mask<G> A = N.ancC & Sub;
            const int y = M.u.piv.stemtab[(A & stem).popc() - 1];
            N.ancC = Ap | (A ^ stem) | Mask<G>::node(y);
            N.potC += dV;
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
        if (l == er) N.bas |= 1ull << ec;
        if (l == lr) N.bas &= ~(1ull << lc);
        if (inC) M.vpot[l] = N.potC;
        wsync();
        ++pivots;
        fresh = false;
        if (theta == 0.0) {
            if (++degenerate_run >= 2 * (T + S)) bland = true;
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
    for (int a = 0; a < T; ++a) sum += M.u.fin.obj[a];
    for (int b = 0; b < S; ++b) sum += M.u.fin.obj[G + b];
    out.d2 = o.want_sqrt ? sqrt(sum) : sum;
    wsync();
    return out;
}

// Dense plan (caller's orientation) and duals of a solved pair.
template <int G>
__device__ void write_certificate(GroupMem<G> &M, const NodeState<G> &N, const PairView &pv, int l,
                                  double *plan, double *duals) {
    const int T = pv.T, S = pv.S;
    const bool hasR = l < T, hasC = l < S;
    M.u.fin.colflow[l] = hasC ? N.flowC : 0.0;
    M.u.fin.colpar[l] = hasC ? N.parC : -1;
    wsync();
    if (plan && hasR) {
        for (int j = 0; j < S; ++j) {
            double w = 0.0;
            if (N.parR == j) w = N.flowR;
            else if (M.u.fin.colpar[j] == l) w = M.u.fin.colflow[j];
            // caller's frame: A side is t x s; rows here are A unless swapped
            int64_t idx = pv.swapped ? ((int64_t)j * T + l) : ((int64_t)l * S + j);
            plan[idx] = w;
        }
    }
    if (duals) {
        // u (A side) then v (B side)
        const int tA = pv.swapped ? S : T;
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

// -------------------------------------------------------------- kernels

template <int G>
struct Cfg {
    static constexpr int waves = G == 16 ? 4 : (G == 32 ? 2 : 1);
    static constexpr int threads = waves * 64;
    static constexpr int groups = threads / G;
};

template <int G, typename TIn>
__global__ __launch_bounds__(Cfg<G>::threads) void k_assign(KSet X, KSet Z, KOpts o, int64_t chunks,
                                                            int64_t per_chunk, int32_t *labels,
                                                            double *best, double *all,
                                                            int32_t *row_status, double *ws_best,
                                                            int32_t *ws_label, int32_t *ws_status) {
    constexpr int NG = Cfg<G>::groups;
    __shared__ GroupMem<G> mem[NG];
    __shared__ double red_v[NG];
    __shared__ int red_i[NG], red_s[NG];
    const int tid = threadIdx.x;
    const int g = tid / G, l = tid % G, gbase = (tid & 63) & ~(G - 1);
    const int64_t total = X.n * chunks;
    const int64_t K = Z.n;
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int64_t i = item / chunks, ch = item % chunks;
        const int64_t j0 = ch * per_chunk;
        const int64_t j1 = j0 + per_chunk < K ? j0 + per_chunk : K;
        double bv = INFINITY;
        int bj = 0x7fffffff, worst = kOk;
        for (int64_t j = j0 + g; j < j1; j += NG) {
            NodeState<G> N;
            PairView pv = orient(X, i, Z, j, (int)sizeof(TIn));
            SolveOut r = solve_pair<G, TIn>(mem[g], N, pv, X.d, o, l, gbase);
            if (r.status != kOk) {
                worst = r.status > worst ? r.status : worst;
                r.d2 = __builtin_nan("");
            } else if (r.d2 < bv || (r.d2 == bv && (int)j < bj)) {
                bv = r.d2;
                bj = (int)j;
            }
            if (all && l == 0) all[i * K + j] = r.d2;
        }
        if (l == 0) { red_v[g] = bv; red_i[g] = bj; red_s[g] = worst; }
        __syncthreads();
        if (tid == 0) {
            double v = INFINITY;
            int jj = 0x7fffffff, st = kOk;
            for (int q = 0; q < NG; ++q) {
                if (red_v[q] < v || (red_v[q] == v && red_i[q] < jj)) { v = red_v[q]; jj = red_i[q]; }
                st = red_s[q] > st ? red_s[q] : st;
            }
            if (chunks == 1) {
                labels[i] = st == kOk ? jj : -1;
                best[i] = st == kOk ? v : __builtin_nan("");
                if (row_status) row_status[i] = st;
            } else {
                ws_best[item] = v;
                ws_label[item] = jj;
                ws_status[item] = st;
            }
        }
        __syncthreads();
    }
}

__global__ void k_assign_reduce(int64_t n, int64_t chunks, const double *ws_best,
                                const int32_t *ws_label, const int32_t *ws_status, int32_t *labels,
                                double *best, int32_t *row_status) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = INFINITY;
    int jj = 0x7fffffff, st = kOk;
    for (int64_t c = 0; c < chunks; ++c) {
        double bv = ws_best[i * chunks + c];
        int bj = ws_label[i * chunks + c];
        if (bv < v || (bv == v && bj < jj)) { v = bv; jj = bj; }
        int s = ws_status[i * chunks + c];
        st = s > st ? s : st;
    }
    labels[i] = st == kOk ? jj : -1;
    best[i] = st == kOk ? v : __builtin_nan("");
    if (row_status) row_status[i] = st;
}

template <int G, typename TIn>
__global__ __launch_bounds__(Cfg<G>::threads) void k_emd_pairs(KSet A, KSet B, const int64_t *pairs,
                                                               int64_t npairs, KOpts o, double *dist,
                                                               const int64_t *plan_off, double *plan,
                                                               const int64_t *dual_off, double *duals,
                                                               int32_t *status) {
    constexpr int NG = Cfg<G>::groups;
    __shared__ GroupMem<G> mem[NG];
    const int tid = threadIdx.x;
    const int g = tid / G, l = tid % G, gbase = (tid & 63) & ~(G - 1);
    const int64_t stride = (int64_t)gridDim.x * NG;
    for (int64_t k = (int64_t)blockIdx.x * NG + g; k < npairs; k += stride) {
        const int64_t i = pairs[2 * k], j = pairs[2 * k + 1];
        int st;
        double val = __builtin_nan("");
        if (i < 0 || i >= A.n || j < 0 || j >= B.n) {
            st = kTooLarge;
        } else {
            NodeState<G> N;
            PairView pv = orient(A, i, B, j, (int)sizeof(TIn));
            SolveOut r = solve_pair<G, TIn>(mem[g], N, pv, A.d, o, l, gbase);
            st = r.status;
            if (st == kOk) {
                val = r.d2;
                if (plan || duals)
                    write_certificate<G>(mem[g], N, pv, l, plan ? plan + plan_off[k] : nullptr,
                                         duals ? duals + dual_off[k] : nullptr);
            }
        }
        if (l == 0) {
            dist[k] = val;
            if (status) status[k] = st;
        }
    }
}

// Row i of the strict upper triangle holds n-1-i pairs; k -> (i, j).
__device__ __forceinline__ void condensed_ij(int64_t n, int64_t k, int64_t &i, int64_t &j) {
    double nn = (double)n;
    double disc = (2.0 * nn - 1.0) * (2.0 * nn - 1.0) - 8.0 * (double)k;
    int64_t r = (int64_t)floor(((2.0 * nn - 1.0) - sqrt(disc > 0.0 ? disc : 0.0)) * 0.5);
    if (r < 0) r = 0;
    if (r > n - 2) r = n - 2;
    // start(r) = r*n - r*(r+1)/2; fix rounding by stepping
    while (r > 0 && r * n - r * (r + 1) / 2 > k) --r;
    while (r + 1 <= n - 2 && (r + 1) * n - (r + 1) * (r + 2) / 2 <= k) ++r;
    i = r;
    j = k - (r * n - r * (r + 1) / 2) + r + 1;
}

template <int G, typename TIn>
__global__ __launch_bounds__(Cfg<G>::threads) void k_pairwise(KSet X, KOpts o, double *out,
                                                              int32_t *status) {
    constexpr int NG = Cfg<G>::groups;
    __shared__ GroupMem<G> mem[NG];
    const int tid = threadIdx.x;
    const int g = tid / G, l = tid % G, gbase = (tid & 63) & ~(G - 1);
    const int64_t m = X.n * (X.n - 1) / 2;
    const int64_t stride = (int64_t)gridDim.x * NG;
    for (int64_t k = (int64_t)blockIdx.x * NG + g; k < m; k += stride) {
        int64_t i, j;
        condensed_ij(X.n, k, i, j);
        NodeState<G> N;
        PairView pv = orient(X, i, X, j, (int)sizeof(TIn));
        SolveOut r = solve_pair<G, TIn>(mem[g], N, pv, X.d, o, l, gbase);
        if (l == 0) {
            out[k] = r.status == kOk ? r.d2 : __builtin_nan("");
            if (status) status[k] = r.status;
        }
    }
}

template <typename TIn>
__global__ void k_cost_tiles_f64(KSet A, KSet B, const int64_t *pairs, int64_t npairs,
                                 double *tiles, const int64_t *tile_off) {
    // one workgroup per pair, threads over cells
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
                double diff = (double)x[a * A.d + q] - (double)y[b * B.d + q];
                acc = fma(diff, diff, acc);
            }
            dst[c] = acc;
        }
    }
}

// ------------------------------------------------------------ launchers

int group_width_for(int maxsup) {
    if (maxsup <= 16) return 16;
    if (maxsup <= 32) return 32;
    return 64;
}

static int groups_per_block(int G) {
    return G == 16 ? Cfg<16>::groups : (G == 32 ? Cfg<32>::groups : Cfg<64>::groups);
}

AssignPlan plan_assign(const KSet &X, const KSet &Z, int maxsup, int cu_count) {
    AssignPlan p;
    p.G = group_width_for(maxsup);
    const int NG = groups_per_block(p.G);
    const int64_t K = Z.n > 0 ? Z.n : 1;
    const int64_t target = (int64_t)(cu_count > 0 ? cu_count : 256) * 8;
    int64_t chunks = X.n > 0 ? (target + X.n - 1) / X.n : 1;
    const int64_t max_chunks = (K + NG - 1) / NG;
    if (chunks > max_chunks) chunks = max_chunks;
    if (chunks < 1) chunks = 1;
    p.chunks = chunks;
    p.per_chunk = (K + chunks - 1) / chunks;
    p.ws_bytes = chunks > 1 ? (size_t)X.n * chunks * (sizeof(double) + 2 * sizeof(int32_t)) : 0;
    return p;
}

template <int G, typename TIn>
static hipError_t assign_t(const LaunchCtx &c, const AssignPlan &p, const KSet &X, const KSet &Z,
                           const KOpts &o, int32_t *labels, double *best, double *all,
                           int32_t *row_status, void *ws) {
    const int64_t total = X.n * p.chunks;
    double *wb = nullptr;
    int32_t *wl = nullptr, *wsn = nullptr;
    if (p.chunks > 1) {
        wb = (double *)ws;
        wl = (int32_t *)(wb + X.n * p.chunks);
        wsn = wl + X.n * p.chunks;
    }
    const int64_t grid = total < (1LL << 30) ? total : (1LL << 30);
    hipLaunchKernelGGL((k_assign<G, TIn>), dim3((unsigned)grid), dim3(Cfg<G>::threads), 0, c.stream, X,
                       Z, o, p.chunks, p.per_chunk, labels, best, all, row_status, wb, wl, wsn);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || p.chunks == 1) return e;
    const int64_t blocks = (X.n + 255) / 256;
    hipLaunchKernelGGL(k_assign_reduce, dim3((unsigned)blocks), dim3(256), 0, c.stream, X.n, p.chunks,
                       wb, wl, wsn, labels, best, row_status);
    return hipGetLastError();
}

hipError_t launch_assign(const LaunchCtx &c, const AssignPlan &p, const KSet &X, const KSet &Z,
                         const KOpts &o, int32_t *labels, double *best, double *all,
                         int32_t *row_status, void *ws) {
    if (X.n == 0) return hipSuccess;
    const bool f32 = X.dtype == D2_F32;
    switch (p.G) {
    case 16: return f32 ? assign_t<16, float>(c, p, X, Z, o, labels, best, all, row_status, ws)
                        : assign_t<16, double>(c, p, X, Z, o, labels, best, all, row_status, ws);
    case 32: return f32 ? assign_t<32, float>(c, p, X, Z, o, labels, best, all, row_status, ws)
                        : assign_t<32, double>(c, p, X, Z, o, labels, best, all, row_status, ws);
    default: return f32 ? assign_t<64, float>(c, p, X, Z, o, labels, best, all, row_status, ws)
                        : assign_t<64, double>(c, p, X, Z, o, labels, best, all, row_status, ws);
    }
}

template <int G, typename TIn>
static hipError_t emd_pairs_t(const LaunchCtx &c, const KSet &A, const KSet &B, const int64_t *pairs,
                              int64_t npairs, const KOpts &o, double *dist, const int64_t *plan_off,
                              double *plan, const int64_t *dual_off, double *duals, int32_t *status) {
    const int NG = Cfg<G>::groups;
    int64_t grid = (npairs + NG - 1) / NG;
    if (grid > (1LL << 30)) grid = 1LL << 30;
    hipLaunchKernelGGL((k_emd_pairs<G, TIn>), dim3((unsigned)grid), dim3(Cfg<G>::threads), 0, c.stream,
                       A, B, pairs, npairs, o, dist, plan_off, plan, dual_off, duals, status);
    return hipGetLastError();
}

hipError_t launch_emd_pairs(const LaunchCtx &c, int G, const KSet &A, const KSet &B,
                            const int64_t *pairs, int64_t npairs, const KOpts &o, double *dist,
                            const int64_t *plan_off, double *plan, const int64_t *dual_off,
                            double *duals, int32_t *status) {
    if (npairs == 0) return hipSuccess;
    const bool f32 = A.dtype == D2_F32;
#define D2_EMD(GG)                                                                                  \
    return f32 ? emd_pairs_t<GG, float>(c, A, B, pairs, npairs, o, dist, plan_off, plan, dual_off,  \
                                        duals, status)                                              \
               : emd_pairs_t<GG, double>(c, A, B, pairs, npairs, o, dist, plan_off, plan, dual_off, \
                                         duals, status)
    switch (G) {
    case 16: D2_EMD(16);
    case 32: D2_EMD(32);
    default: D2_EMD(64);
    }
#undef D2_EMD
}

template <int G, typename TIn>
static hipError_t pairwise_t(const LaunchCtx &c, const KSet &X, const KOpts &o, double *out,
                             int32_t *status) {
    const int NG = Cfg<G>::groups;
    const int64_t m = X.n * (X.n - 1) / 2;
    int64_t grid = (m + NG - 1) / NG;
    if (grid > (1LL << 30)) grid = 1LL << 30;
    hipLaunchKernelGGL((k_pairwise<G, TIn>), dim3((unsigned)grid), dim3(Cfg<G>::threads), 0, c.stream,
                       X, o, out, status);
    return hipGetLastError();
}

hipError_t launch_pairwise(const LaunchCtx &c, int G, const KSet &X, const KOpts &o,
                           double *condensed, int32_t *status) {
    if (X.n < 2) return hipSuccess;
    const bool f32 = X.dtype == D2_F32;
    switch (G) {
    case 16: return f32 ? pairwise_t<16, float>(c, X, o, condensed, status)
                        : pairwise_t<16, double>(c, X, o, condensed, status);
    case 32: return f32 ? pairwise_t<32, float>(c, X, o, condensed, status)
                        : pairwise_t<32, double>(c, X, o, condensed, status);
    default: return f32 ? pairwise_t<64, float>(c, X, o, condensed, status)
                        : pairwise_t<64, double>(c, X, o, condensed, status);
    }
}

hipError_t launch_cost_tiles(const LaunchCtx &c, const KSet &A, const KSet &B,
                             const int64_t *pairs, int64_t npairs, int cost_mode, double *tiles,
                             const int64_t *tile_off) {
    if (npairs == 0) return hipSuccess;
    (void)cost_mode;
    int64_t grid = npairs < (1LL << 30) ? npairs : (1LL << 30);
    if (A.dtype == D2_F32)
        hipLaunchKernelGGL(k_cost_tiles_f64<float>, dim3((unsigned)grid), dim3(256), 0, c.stream, A, B,
                           pairs, npairs, tiles, tile_off);
    else
        hipLaunchKernelGGL(k_cost_tiles_f64<double>, dim3((unsigned)grid), dim3(256), 0, c.stream, A, B,
                           pairs, npairs, tiles, tile_off);
    return hipGetLastError();
}

}  // namespace d2
