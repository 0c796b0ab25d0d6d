// D^2 for an explicit pair list with each pair's optimal basis as a list of
// cells: the t + s - 1 edges of the spanning tree that the transportation
// simplex ends on (Sec. 1.1: for fixed centroid atoms the LP of Eq. (1) is
// a transportation problem, whose bases are spanning trees of the bipartite
// graph of the two atom sets).  The solver is the same inlined lane-group
// solver as every other entry point; only the output differs from the dense
// plan of d2_emd_batch.  Cells are written sorted by (A atom, B atom), in
// the caller's orientation, zero-flow (degenerate) basic cells included.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "d2_internal.h"
#include "d2_shapes.h"
#include "d2_solver.h"

namespace d2 {

namespace {

// The tree's edges of one solved pair, as (A atom, B atom, flow) cells.
// Every lane publishes the parent edge of its row node and of its column
// node; then lane l takes the caller's A atom l (a solver row, or a solver
// column when the pair was swapped): its own parent edge and the edges of
// the other side's nodes whose parent it is, in ascending B atom order,
// after the cells of the atoms before it.
template <int G, int GS, bool LT>
__device__ __forceinline__ void write_basis(GroupMem<G, GS> &M, const NodeState<G, GS, LT> &N,
                                            const PairView &pv, int l, int32_t *ij, double *w) {
    const int T = pv.T, S = pv.S;
    const bool hasR = l < T, hasC = l < S;
    int *par = M.u.piv.newpar;        // [0, G): rows' parent columns; [G, G + GS): columns' parent rows
    double *flow = M.u.piv.newflow;
    int *cnt = M.u.piv.stemtab;       // cells of each A atom
    par[l] = hasR ? N.parR : -1;
    flow[l] = hasR ? N.flowR : 0.0;
    if (l < GS) {
        par[G + l] = hasC ? N.parC : -1;
        flow[G + l] = hasC ? N.flowC : 0.0;
    }
    wsync();
    // A side: solver rows unless swapped
    const int na = pv.swapped ? S : T, nb = pv.swapped ? T : S;
    const int own = pv.swapped ? G : 0, other = pv.swapped ? 0 : G;
    const bool mine = l < na;
    int c = 0;
    if (mine) {
        c = par[own + l] >= 0 ? 1 : 0;
        for (int x = 0; x < nb; ++x) c += par[other + x] == l ? 1 : 0;
        cnt[l] = c;
    }
    wsync();
    if (mine) {
        int pos = 0;
        for (int q = 0; q < l; ++q) pos += cnt[q];
        const int p = par[own + l];
        for (int x = 0; x < nb; ++x) {
            double f;
            if (x == p) f = flow[own + l];
            else if (par[other + x] == l) f = flow[other + x];
            else continue;
            ij[2 * pos] = l;
            ij[2 * pos + 1] = x;
            w[pos] = f;
            ++pos;
        }
    }
    wsync();
}

template <int CLS, typename TIn, int START>
__global__ __launch_bounds__(ShapeCfg<CLS>::threads, ShapeCfg<CLS>::occ) void k_emd_basis(
    KSet A, KSet B, const int64_t *pairs, int64_t npairs, KOpts o, double *dist, const int64_t *basis_off,
    int32_t *basis_ij, double *basis_w, int32_t *status) {
    constexpr int G = ShapeCfg<CLS>::G, GS = ShapeCfg<CLS>::GS, NG = ShapeCfg<CLS>::groups;
    constexpr bool LT = ShapeCfg<CLS>::LT;
    __shared__ GroupMem<G, GS> mem[NG];
    __shared__ TileOf<CLS, START> tiles[NG];
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
            NodeState<G, GS, LT> N;
            PairView pv = orient(A, i, B, j, (int)sizeof(TIn));
            SolveOut r = solve_pair<G, GS, LT, TIn, START>(mem[g], tiles[g], N, pv, A.d, o, l, gbase);
            st = r.status;
            if (st == kOk) {
                val = r.d2;
                write_basis<G, GS, LT>(mem[g], N, pv, l, basis_ij + 2 * basis_off[k], basis_w + basis_off[k]);
            }
        }
        if (l == 0) {
            dist[k] = val;
            if (status) status[k] = st;
        }
    }
}

struct BasisRun {
    const LaunchCtx &c;
    const KSet &A, &B;
    const int64_t *pairs; int64_t npairs;
    const KOpts &o;
    double *dist; const int64_t *basis_off; int32_t *basis_ij; double *basis_w; int32_t *status;
    template <int C, typename TIn, int V>
    hipError_t run() {
        const int NG = ShapeCfg<C>::groups;
        int64_t grid = (npairs + NG - 1) / NG;
        if (grid > (1LL << 30)) grid = 1LL << 30;
        hipLaunchKernelGGL((k_emd_basis<C, TIn, V>), dim3((unsigned)grid), dim3(ShapeCfg<C>::threads), 0,
                           c.stream, A, B, pairs, npairs, o, dist, basis_off, basis_ij, basis_w, status);
        return hipGetLastError();
    }
};

}  // namespace

hipError_t launch_emd_basis(const LaunchCtx &c, int cls, const KSet &A, const KSet &B, const int64_t *pairs,
                            int64_t npairs, const KOpts &o, double *dist, const int64_t *basis_off,
                            int32_t *basis_ij, double *basis_w, int32_t *status) {
    if (npairs == 0) return hipSuccess;
    BasisRun r{c, A, B, pairs, npairs, o, dist, basis_off, basis_ij, basis_w, status};
    return dispatch_class(cls, A.dtype == D2_F32, o.init, r);
}

}  // namespace d2
