// The transport LP of Eq. (1) over caller-given ground costs: the same
// solver, with cost rows loaded from an FP64 matrix instead of computed from
// points.  It serves the MM distance of Eq. (10), whose ground cost is a
// matrix of squared Mallows distances between centroids, and any other cost
// a caller has.
//
// Problem k: row weights rw[roff[k] .. roff[k+1]), column weights
// cw[coff[k] .. coff[k+1]), cost matrix at cost + moff[k], row-major
// t_k x s_k.  The pair is oriented as every other pair (rows = the larger
// side); when that swaps the sides, the cost is read transposed and the plan
// written back in the caller's frame.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "d2_internal.h"
#include "d2_shapes.h"
#include "d2_solver.h"

namespace d2 {

namespace {

template <int CLS, int START>
__global__ __launch_bounds__(ShapeCfg<CLS>::threads, ShapeCfg<CLS>::occ) void k_emd_cost(
    int64_t nprob, const int64_t *roff, const double *rw, const int64_t *coff, const double *cw,
    const double *cost, const int64_t *moff, int max_rows, int max_cols, KOpts o, double *dist,
    const int64_t *plan_off, double *plan, int32_t *status) {
    constexpr int G = ShapeCfg<CLS>::G, GS = ShapeCfg<CLS>::GS, NG = ShapeCfg<CLS>::groups;
    constexpr bool LT = ShapeCfg<CLS>::LT;
    using TileT = TileOf<CLS, START>;
    __shared__ GroupMem<G, GS> mem[NG];
    __shared__ TileT tiles[NG];
    const int tid = threadIdx.x;
    const int g = tid / G, l = tid % G, gbase = (tid & 63) & ~(G - 1);
    const int64_t stride = (int64_t)gridDim.x * NG;
    for (int64_t k = (int64_t)blockIdx.x * NG + g; k < nprob; k += stride) {
        const int64_t r0 = roff[k], c0 = coff[k];
        const int64_t t = roff[k + 1] - r0, s = coff[k + 1] - c0;
        SolveOut r{kTooLarge, __builtin_nan("")};
        NodeState<G, GS, LT> N;
        PairView pv;
        pv.xr = nullptr;
        pv.xc = nullptr;
        int64_t grs, gcs;
        if (t >= s) {
            pv.wr = rw + r0; pv.T = (int)(t < 0 ? 0 : t);
            pv.wc = cw + c0; pv.S = (int)(s < 0 ? 0 : s);
            pv.swapped = false;
            grs = s; gcs = 1;
        } else {
            pv.wr = cw + c0; pv.T = (int)(s < 0 ? 0 : s);
            pv.wc = rw + r0; pv.S = (int)(t < 0 ? 0 : t);
            pv.swapped = true;
            grs = 1; gcs = s;
        }
        // uniform over the group; the declared bounds size the caller's plan
        if (t >= 1 && s >= 1 && t <= max_rows && s <= max_cols)
            r = solve_pair<G, GS, LT, double, START, TileT, true>(mem[g], tiles[g], N, pv, 1, o, l, gbase,
                                                                  cost + moff[k], grs, gcs);
        if (r.status == kOk && plan)
            write_certificate<G, GS, LT>(mem[g], N, pv, l, plan + plan_off[k], nullptr);
        if (l == 0) {
            dist[k] = r.status == kOk ? r.d2 : __builtin_nan("");
            if (status) status[k] = r.status;
        }
    }
}

struct CostRun {
    const LaunchCtx &c;
    int64_t nprob;
    const int64_t *roff; const double *rw; const int64_t *coff; const double *cw;
    const double *cost; const int64_t *moff;
    int max_rows, max_cols;
    const KOpts &o;
    double *dist; const int64_t *plan_off; double *plan; int32_t *status;
    template <int C, typename TIn, int V>
    hipError_t run() {
        const int NG = ShapeCfg<C>::groups;
        int64_t grid = (nprob + NG - 1) / NG;
        if (grid > (1LL << 30)) grid = 1LL << 30;
        hipLaunchKernelGGL((k_emd_cost<C, V>), dim3((unsigned)grid), dim3(ShapeCfg<C>::threads), 0, c.stream,
                           nprob, roff, rw, coff, cw, cost, moff, max_rows, max_cols, o, dist, plan_off, plan,
                           status);
        return hipGetLastError();
    }
};

}  // namespace

hipError_t launch_emd_cost(const LaunchCtx &c, int cls, int64_t nprob, const int64_t *roff, const double *rw,
                           const int64_t *coff, const double *cw, const double *cost, const int64_t *moff,
                           int max_rows, int max_cols, const KOpts &o, double *dist, const int64_t *plan_off,
                           double *plan, int32_t *status) {
    if (nprob == 0) return hipSuccess;
    CostRun r{c, nprob, roff, rw, coff, cw, cost, moff, max_rows, max_cols, o, dist, plan_off, plan, status};
    return dispatch_class(cls, false, o.init, r);
}

}  // namespace d2
